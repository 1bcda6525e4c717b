// Reference Philox4x32-10 taken from rocRAND's engine (an independent library
// implementation), used only to pin the oracle's generator.  The engine is seeded with
// key = seed and positioned at counter (x, y, z, w) through its subsequence (z, w) and
// offset (4 * (x | y << 32)) arguments; next4() then returns Philox(counter, key).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void ref_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t* c = ctr + 4 * i;
    unsigned long long seed = (unsigned long long)key[0] | ((unsigned long long)key[1] << 32);
    unsigned long long subseq = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
    unsigned long long offset = 4ull * ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
    uint4 r = eng.next4();
    out[4 * i + 0] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
  }
}
