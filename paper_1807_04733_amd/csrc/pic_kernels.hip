// Device kernels of the hot-electron particle-in-cell step for gfx950 (CDNA4, wave64).
//
// One launch of k_step advances every carrier of every instance by one step of the
// Strang splitting of arXiv:1807.04733 Eq. (15):
//   Source(dt/2)     primaries scheduled for this step are created in registers (Eq. 17)
//   Transport(dt/2)  straight flight, vacuum reflection, stochastic interfaces (Eq. 18)
//   Scattering(dt)   Monte-Carlo event with p = 1 - exp(-dt/tau_eff) (Eq. 2, Sec. III.A):
//                    elastic (Eq. 8) or inelastic with an energy-conserving secondary
//                    (Eqs. 6-7, 19); products below E_min are removed
//   Transport(dt/2)  for the survivor and the newborn
//   deposit          density and v*cos(theta) moments (Eqs. 16, 23) into LDS histograms
//
// Data layout: structure-of-arrays particle state streamed once per step (z, cos(theta),
// energy, uid, flags), partitioned into slabs that each belong to one instance.  A slab
// is processed by one workgroup per step, which appends newborns behind the slab's tail
// with a wave ballot + one LDS atomic per wave (no global atomics on the append path).
// Histograms are privatised per workgroup in LDS and merged into the int64 bins with
// global atomics only for non-zero entries.  All decisions use binary64 arithmetic in
// the order written here; the file is built with -ffp-contract=off.
#include "pic_device.h"

#pragma clang fp contract(off)

namespace pic {

// Compile-time launch modes of the step kernel.
constexpr int kModeDebug = 1;       // keep per-particle event counts
constexpr int kModeDensLds = 2;     // this step deposits density into LDS
constexpr int kModeDensGlobal = 4;  // this step deposits density with global atomics
constexpr int kModeCur = 8;         // this step deposits the current

template <int MODE>
__device__ __forceinline__ void deposit(const StepArgs& a, const DevInst& I, uint32_t* s_dens,
                                        unsigned long long* s_cur, const uint32_t* s_edges,
                                        double z, double mu, uint32_t E, uint32_t fl, double v) {
  int zb = (int)floor(z * I.inv_dz);
  zb = zb < 0 ? 0 : (zb > I.nz - 1 ? I.nz - 1 : zb);
  const int s = (int)(fl & kSpinMask);
  if (MODE & (kModeDensLds | kModeDensGlobal)) {
    const int eb = a.n_ebins > 1 ? energy_bin(s_edges, a.n_ebins, E) : 0;
    const int idx = (zb * a.n_ebins + eb) * 2 + s;
    if (MODE & kModeDensLds) {
      atomicAdd(&s_dens[idx], 1u);
    } else {
      const int64_t g = I.dens_off + (int64_t)a.dens_slot * I.nz * a.n_ebins * 2 + idx;
      atomicAdd((unsigned long long*)&a.dens[g], 1ull);
    }
  }
  if (MODE & kModeCur) {
    const double vm = v * mu;
    // round-half-even to an integer by adding 1.5*2^52 (|vm*2^32| < 2^51): the low
    // mantissa bits then hold the integer, identical to rint()
    const double sh = vm * 4294967296.0 + 0x1.8p52;
    const long long val = __double_as_longlong(sh) - __double_as_longlong(0x1.8p52);
    atomicAdd(&s_cur[zb * 2 + s], (unsigned long long)val);
  }
}

template <int MODE>
__device__ void flush_bins(const StepArgs& a, const DevInst& I, uint32_t* s_dens,
                           unsigned long long* s_cur) {
  __syncthreads();
  if (MODE & kModeDensLds) {
    const int n = I.nz * a.n_ebins * 2;
    unsigned long long* g =
        (unsigned long long*)(a.dens + I.dens_off + (int64_t)a.dens_slot * n);
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
      const uint32_t v = s_dens[b];
      if (v) {
        atomicAdd(&g[b], (unsigned long long)v);
        s_dens[b] = 0;
      }
    }
  }
  if (MODE & kModeCur) {
    const int n = I.nz * 2;
    unsigned long long* g = (unsigned long long*)(a.cur + I.cur_off + (int64_t)a.cur_slot * n);
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
      const unsigned long long v = s_cur[b];
      if (v) {
        atomicAdd(&g[b], v);
        s_cur[b] = 0;
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void wave_add(unsigned long long* c, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    if (__lane_id() == leader) atomicAdd(c, (unsigned long long)__popcll(m));
  }
}

// Newborn secondaries wait in a wave-private LDS queue and are finished 64 at a time, so
// the spawn draw, the newborn's half step, its deposit and its append run as full
// waves instead of once per wave for a few lanes.
constexpr int kQ = 128;
struct ChildQueue {  // kChildQueueBytes
  double z[kQ];
  uint32_t lo[kQ], hi[kQ], E[kQ], fl[kQ];
};

// The SoA arrays offset to one slab: uniform base pointers with 32-bit lane offsets.
template <typename F>
struct SlabPtrs {
  F* z;
  F* mu;
  uint32_t* E;
  uint64_t* uid;
  uint32_t* fl;
  uint64_t* ev;
};

struct LaneCounts {
  uint32_t dep, tr, ri, rs;
};

// Finish the top n entries of a wave's queue: spawn draw (direction, spin from the
// layer's equilibrium polarisation, lineage), second half step, deposit and append.
template <typename F, int MODE>
__device__ __forceinline__ void drain_children(const StepArgs& a, const DevInst& I, ChildQueue& Q,
                                               int qn, int n, uint32_t* s_dens,
                                               unsigned long long* s_cur, const uint32_t* s_edges,
                                               int* s_app, const SlabPtrs<F>& sp, int tail0,
                                               int cap, LaneCounts& lc, bool& bad) {
  constexpr bool DEBUG = (MODE & kModeDebug) != 0;
  const int lane = __lane_id();
  const bool act = lane < n;
  const int idx = act ? qn - n + lane : 0;
  double cz = Q.z[idx];
  const uint32_t lo = Q.lo[idx], phi = Q.hi[idx], cE = Q.E[idx], pfl = Q.fl[idx];
  if (act) {
    const uint4 sw = philox10(lo, phi, (uint32_t)a.step, kTagSpawn, a.key0, a.key1);
    const int l = layer_of(pfl);
    double cmu = to_store<F>(dircos(sw.x));
    const uint32_t cs = u01(sw.y) < I.lay[l].w ? 0u : 1u;
    uint32_t lin = sw.z;
    if (lin == 0u || lin == phi) {
      lin = sw.w | 1u;
      if (lin == phi) lin ^= 2u;
    }
    const uint32_t z_next = a.z_write ? 0u : (uint32_t)a.z_phase + 1u;
    uint32_t cfl = cs | (pfl & ~kSpinMask) | (z_next << kStampShift);
    HitCounts h{0, 0, 0};
    LayCache cc = load_lay(I, l, (int)cs);
    half_push_c(I, cc, cz, cmu, cfl, cE, lo, lin, (uint32_t)a.step, kTagHalf2, a.h, a.key0,
                a.key1, h, bad);
    cz = to_store<F>(cz);
    deposit<MODE>(a, I, s_dens, s_cur, s_edges, cz, cmu, cE, cfl, cc.v);
    lc.dep += 1;
    lc.tr += h.tr;
    lc.ri += h.ri;
    lc.rs += h.rs;
    const uint64_t m = __ballot(1);
    int off = 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    if (lane == leader) off = atomicAdd(s_app, __popcll(m));
    off = __shfl(off, leader);
    const uint32_t pos = (uint32_t)(tail0 + off + prefix_count(m));
    if ((int)pos < cap) {
      sp.z[pos] = (F)cz;
      sp.mu[pos] = (F)cmu;
      sp.E[pos] = cE;
      sp.uid[pos] = (uint64_t)lo | ((uint64_t)lin << 32);
      sp.fl[pos] = cfl;
      if (DEBUG) sp.ev[pos] = ((uint64_t)h.tr << 16) + ((uint64_t)(h.ri + h.rs) << 32);
    } else {
      atomicOr(a.status, kStOverflow);
    }
  }
}

// Slots whose step needs the general path (a boundary hit, or a draw below x that may be
// an event) wait in a wave-private LDS queue; their state is still untouched in HBM and
// is re-read when 64 have gathered, so the general path runs as full waves while the
// common step (no hit, certainly no event) runs without divergent branches.
constexpr int kSlowQ = 128;

template <typename F, int MODE>
__global__ void __launch_bounds__(512, 4) k_step(StepArgs a) {
  constexpr bool DEBUG = (MODE & kModeDebug) != 0;
  // dynamic LDS: [density histogram | current histogram | child queue per wave |
  //               general-path slot queue per wave]
  extern __shared__ __align__(16) unsigned char dyn[];
  uint32_t* s_dens = (uint32_t*)dyn;
  const size_t cur_at = ((size_t)a.lds_dens_words * 4 + 15) & ~(size_t)15;
  unsigned long long* s_cur = (unsigned long long*)(dyn + cur_at);
  const size_t q_at = (cur_at + (size_t)a.lds_cur_words * 8 + 15) & ~(size_t)15;
  ChildQueue* s_q = (ChildQueue*)(dyn + q_at);
  uint32_t* s_slow = (uint32_t*)(dyn + q_at + (size_t)(blockDim.x >> 6) * kChildQueueBytes);
  __shared__ DevInst s_inst;
  __shared__ unsigned long long s_cnt[kNC];
  __shared__ uint32_t s_edges[PIC_MAX_EBINS];
  __shared__ int s_slab, s_app, s_dead;
  __shared__ unsigned long long s_fast, s_left;

  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int wave = tid >> 6;
  if (tid == 0) {
    s_fast = 0;
    s_left = 0;
  }
  uint32_t n_fast = 0, n_left = 0;
  for (int i = tid; i < a.lds_dens_words; i += blockDim.x) s_dens[i] = 0;
  for (int i = tid; i < a.lds_cur_words; i += blockDim.x) s_cur[i] = 0;
  for (int i = tid; i < a.n_ebins; i += blockDim.x) s_edges[i] = a.e_edges[i];
  if (tid < kNC) s_cnt[tid] = 0;

  F* gz = (F*)a.z;
  F* gmu = (F*)a.mu;
  const uint32_t step = (uint32_t)a.step;
  // stamp of every z this step stores (0 when the step ends a write-back period)
  const uint32_t z_next = a.z_write ? 0u : (uint32_t)a.z_phase + 1u;
  ChildQueue& Q = s_q[wave];
  uint32_t* SQ = s_slow + wave * kSlowQ;
  static_assert(sizeof(ChildQueue) == kChildQueueBytes, "queue layout");
  int cur_inst = -1;
  bool bad = false;

  for (;;) {
    if (tid == 0) s_slab = atomicAdd(&a.queue[a.step], 1);
    __syncthreads();
    const int slab = s_slab;
    if (slab >= a.n_slabs) break;
    const int inst = a.slab_inst[slab];
    if (inst != cur_inst) {
      if (cur_inst >= 0) flush_bins<MODE>(a, s_inst, s_dens, s_cur);
      const uint4* src = (const uint4*)&a.inst[inst];
      uint4* dst = (uint4*)&s_inst;
      for (int i = tid; i < a.inst_bytes / 16; i += blockDim.x) dst[i] = src[i];
      cur_inst = inst;
    }
    if (tid == 0) {
      s_app = 0;
      s_dead = 0;
    }
    __syncthreads();
    const DevInst& I = s_inst;
    const int64_t base = a.slab_base[slab];
    const int cap = a.slab_cap[slab];
    const int tail0 = a.slab_tail[slab];
    const int64_t kk = a.slab_k[slab];
    const int64_t S = I.n_slabs;
    const int64_t* cum = a.inj_cum + (int64_t)inst * (a.n_steps + 1);
    const int64_t f0 = count_mod(cum[step], kk, S);
    const int n_inj = (int)(count_mod(cum[step + 1], kk, S) - f0);
    const int total = tail0 + n_inj;
    if (tid == 0 && n_inj) atomicAdd(&s_cnt[PIC_C_INJECTED], (unsigned long long)n_inj);
    const SlabPtrs<F> sp{gz + base, gmu + base, a.E + base, a.uid + base, a.flags + base,
                         DEBUG ? a.ev + base : nullptr};
    LaneCounts lc{0, 0, 0, 0};
    int qn = 0;  // wave-uniform fill of this wave's child queue
    int sn = 0;  // wave-uniform fill of this wave's general-path queue

    // ---------------------------------------------------------------- general path
    // The whole step for one carrier: boundary hits, the exact scattering decision,
    // elastic / inelastic events, absorption, the newborn's queueing, the append of a
    // new primary and the write-back.  All lanes of the wave call it together; lanes
    // with nothing to do pass a dead carrier.
    auto general = [&](bool from_soa, bool is_new, uint32_t gi, double z, double mu,
                       uint32_t E, uint32_t fl, uint32_t lo, uint32_t hi, uint64_t evp) {
      const bool alive0 = !(fl & kDead);
      bool died = false, spawn = false;
      uint32_t dirty = 0;  // 1: mu, 2: E, 4: flags
      double zmid = 0.0;
      uint32_t E2 = 0, flmid = 0;
      HitCounts hc{0, 0, 0};
      if (alive0) {
        const double mu_in = mu;
        const uint32_t fl_in = fl;
        LayCache c = load_lay(I, layer_of(fl), (int)(fl & kSpinMask));
        half_push_c(I, c, z, mu, fl, E, lo, hi, step, kTagHalf1, a.h, a.key0, a.key1, hc, bad);
        // ---- scattering over the full step, at the mid-step state
        const uint4 w = philox10(lo, hi, step, kTagScat, a.key0, a.key1);
        const double E_ev = (double)E * 0x1p-30;
        const double Ek = a.tau_exp2 ? E_ev * E_ev : 1.0;
        const double itel = I.lay[layer_of(fl)].z;
        const double rate = Ek * c.itau + itel;
        const double x = a.dt * rate;
        const double u0 = u01(w.x);
        // event iff u0 < p = 1 - exp(-x), decided without the transcendental outside a
        // sliver: x - x^2/2 < p < x, with a margin (about x^3/6) far above rounding
        bool event;
        if (u0 >= x) {
          event = false;
        } else if (x >= 0x1p-20 && u0 < x - 0.5 * x * x) {
          event = true;
        } else {
          event = u0 < -expm1(-x);
        }
        if (event) {
          if (DEBUG) evp += 1ull;
          const bool elastic = itel > 0.0 && u01(w.y) < itel / rate;
          mu = to_store<F>(dircos(w.z));
          dirty |= 1u;
          if (elastic) {
            atomicAdd(&s_cnt[PIC_C_EV_EL], 1ull);
          } else {
            atomicAdd(&s_cnt[PIC_C_EV_EE], 1ull);
            const uint32_t E1 = __umulhi(w.w, E);
            E2 = E - E1;
            E = E1;
            dirty |= 2u;
            if (a.secondaries) {
              if (E2 >= a.e_min) {
                spawn = true;
                zmid = z;
                flmid = fl;
                if (DEBUG) evp += 1ull << 48;
                atomicAdd(&s_cnt[PIC_C_SPAWNED], 1ull);
              } else {
                atomicAdd(&s_cnt[PIC_C_SEC_ABSORBED], 1ull);
                atomicAdd(&s_cnt[PIC_C_E_ABSORBED], (unsigned long long)E2);
              }
            }
            if (E1 < a.e_min) {
              died = true;
              atomicAdd(&s_cnt[PIC_C_ABSORBED], 1ull);
              atomicAdd(&s_cnt[PIC_C_E_ABSORBED], (unsigned long long)E1);
            }
          }
        }
        if (!died) {
          half_push_c(I, c, z, mu, fl, E, lo, hi, step, kTagHalf2, a.h, a.key0, a.key1, hc, bad);
          z = to_store<F>(z);
          deposit<MODE>(a, I, s_dens, s_cur, s_edges, z, mu, E, fl, c.v);
          lc.dep += 1;
        } else {
          z = to_store<F>(z);
          fl |= kDead;
        }
        // z is stored below: the stamp says at which step of the write-back period
        fl = (fl & ~(kStampMask << kStampShift)) | (died ? 0u : z_next << kStampShift);
        if (mu != mu_in) dirty |= 1u;
        if (fl != fl_in) dirty |= 4u;
        if (DEBUG) evp += ((uint64_t)hc.tr << 16) + ((uint64_t)(hc.ri + hc.rs) << 32);
      }
      lc.tr += hc.tr;
      lc.ri += hc.ri;
      lc.rs += hc.rs;

      // ---- queue the newborns: (mid-step position, parent uid, energy, layer | gen)
      const uint64_t mq = __ballot(spawn);
      if (mq) {
        if (spawn) {
          const int p = qn + prefix_count(mq);
          uint32_t gen = (flmid >> kGenShift) & kGenMask;
          gen = gen < 255u ? gen + 1u : 255u;
          Q.z[p] = zmid;
          Q.lo[p] = lo;
          Q.hi[p] = hi;
          Q.E[p] = E2;
          Q.fl[p] = (flmid & (kLayerMask << kLayerShift)) | (gen << kGenShift);
        }
        qn += __popcll(mq);
      }
      // ---- append the new primary (always, so that an absorbed one leaves its record)
      const uint64_t ma = __ballot(is_new);
      if (ma) {
        int off = 0;
        const int leader = __ffsll((unsigned long long)ma) - 1;
        if (lane == leader) off = atomicAdd(&s_app, __popcll(ma));
        off = __shfl(off, leader);
        if (is_new) {
          const uint32_t pos = (uint32_t)(tail0 + off + prefix_count(ma));
          if ((int)pos < cap) {
            sp.z[pos] = (F)z;
            sp.mu[pos] = (F)mu;
            sp.E[pos] = E;
            sp.uid[pos] = (uint64_t)lo | ((uint64_t)hi << 32);
            sp.fl[pos] = fl;
            if (DEBUG) sp.ev[pos] = evp;
          } else {
            atomicOr(a.status, kStOverflow);
          }
        }
      }
      if (from_soa && alive0) {
        sp.z[gi] = (F)z;
        if (dirty & 1u) sp.mu[gi] = (F)mu;
        if (dirty & 2u) sp.E[gi] = E;
        if (dirty & 4u) sp.fl[gi] = fl;
        if (DEBUG) sp.ev[gi] = evp;
      }
      const uint64_t md = __ballot(died);
      if (md && lane == __ffsll((unsigned long long)md) - 1) atomicAdd(&s_dead, __popcll(md));
    };

    auto wave_sync = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // finish the top n queued general-path slots (state re-read from HBM)
    auto drain_slow = [&](int n) {
      wave_sync();
      const bool act = lane < n;
      const uint32_t g = act ? SQ[sn - n + lane] : 0u;
      sn -= n;
      uint32_t fl = kDead, E = 0, lo = 0, hi = 0;
      double z = 0.0, mu = 0.0;
      uint64_t evp = 0;
      if (act) {
        fl = sp.fl[g];
        z = (double)sp.z[g];
        mu = (double)sp.mu[g];
        E = sp.E[g];
        const uint64_t u = sp.uid[g];
        lo = (uint32_t)u;
        hi = (uint32_t)(u >> 32);
        if (DEBUG) evp = sp.ev[g];
        const int d = a.z_phase - (int)((fl >> kStampShift) & kStampMask);
        if (d > 0) {
          const LayCache c = load_lay(I, layer_of(fl), (int)(fl & kSpinMask));
          z = replay_flights<F>(z, (c.v * mu) * a.h, d);
        }
      }
      general(act, false, g, z, mu, E, fl, lo, hi, evp);
      wave_sync();
    };
    auto drain_kids = [&](int n) {
      wave_sync();
      drain_children<F, MODE>(a, I, Q, qn, n, s_dens, s_cur, s_edges, &s_app, sp, tail0, cap,
                              lc, bad);
      qn -= n;
      wave_sync();
    };

    // The slot a lane will handle in its next iteration is fetched one iteration ahead,
    // unconditionally (a dead slot's fields are loaded too), so that no load waits on
    // another and each wave keeps two particles' worth of loads in flight.
    F nz = 0, nmu = 0;
    uint32_t nE = 0, nfl = kDead;
    uint64_t nu = 0;
    auto fetch = [&](int t) {
      if (t < tail0) {
        const uint32_t g = (uint32_t)t;
        nfl = sp.fl[g];
        nz = sp.z[g];
        nmu = sp.mu[g];
        nE = sp.E[g];
        nu = sp.uid[g];
      } else {
        nfl = kDead;
      }
    };
    fetch(wave * 64 + lane);
    for (int tb = wave * 64; tb < total; tb += blockDim.x) {
      const int t = tb + lane;
      const F rz = nz, rmu = nmu;
      const uint32_t rE = nE, rfl = nfl;
      const uint64_t ru = nu;
      fetch(t + (int)blockDim.x);
      const bool have = t < total;
      const bool from_soa = have && t < tail0;
      const bool is_new = have && !from_soa;
      const uint32_t gi = (uint32_t)t;

      // ---- common step: no boundary in either half step and a draw at or above
      // x >= p, so certainly no event; identical arithmetic to the general path
      bool slow = false;
      if (from_soa && !(rfl & kDead)) {
        const int l = layer_of(rfl), s = (int)(rfl & kSpinMask);
        const LayCache c = load_lay(I, l, s);
        const double mu = (double)rmu;
        const uint32_t st = (rfl >> kStampShift) & kStampMask;
        const double z0 = replay_flights<F>((double)rz, (c.v * mu) * a.h, a.z_phase - (int)st);
        const double zm = z0 + (c.v * mu) * a.h;
        const uint4 w = philox10((uint32_t)ru, (uint32_t)(ru >> 32), step, kTagScat, a.key0,
                                 a.key1);
        const double E_ev = (double)rE * 0x1p-30;
        const double Ek = a.tau_exp2 ? E_ev * E_ev : 1.0;
        const double x = a.dt * (Ek * c.itau + I.lay[l].z);
        const double ze = zm + (c.v * mu) * a.h;
        slow = zm > c.zhi || zm < c.zlo || u01(w.x) < x || ze > c.zhi || ze < c.zlo;
        if (!slow) {
          const double zs = to_store<F>(ze);
          deposit<MODE>(a, I, s_dens, s_cur, s_edges, zs, mu, rE, rfl, c.v);
          if (a.z_write) {
            sp.z[gi] = (F)zs;
            if (st) sp.fl[gi] = rfl & ~(kStampMask << kStampShift);
          }
          lc.dep += 1;
          n_fast += 1;
        } else {
          n_left += 1;
        }
      }
      // ---- new primaries (source term, Eq. 17) take the general path at once
      if (__ballot(is_new)) {
        double z = 0.0, mu = 0.0;
        uint32_t E = 0, fl = kDead, lo = 0;
        if (is_new) {
          const int64_t j = kk + S * (f0 + (t - tail0));
          const uint32_t root = (uint32_t)(I.root_offset + (uint64_t)j);
          const uint4 w = philox10(root, 0u, 0xFFFFFFFFu, kTagInject, a.key0, a.key1);
          double z0;
          if (I.src_lambda > 0.0)
            z0 = I.src_lo - I.src_lambda * log1p(-u01(w.x) * I.src_cd);
          else
            z0 = I.src_lo + u01(w.x) * (I.src_hi - I.src_lo);
          z = to_store<F>(z0);
          mu = to_store<F>(dircos(w.y));
          const uint32_t s = u01(w.z) < I.src_up ? 0u : 1u;
          E = I.e_lo[s] + __umulhi(w.w, I.e_span[s]);
          int l = 0;
          for (int q = 1; q < I.n_layers; ++q)
            if (I.lay[q].x <= z) l = q;
          fl = s | ((uint32_t)l << kLayerShift) | (1u << kGenShift);
          lo = root;
        }
        general(false, is_new, gi, z, mu, E, fl, lo, 0u, 0ull);
        if (qn >= 64) drain_kids(64);
      }
      // ---- queue the general-path slots; each general pass adds at most 64 newborns,
      // so the newborn queue (128) is drained below 64 before every pass
      const uint64_t ms = __ballot(slow);
      if (ms) {
        if (slow) SQ[sn + prefix_count(ms)] = gi;
        sn += __popcll(ms);
      }
      if (sn >= 64) {
        drain_slow(64);
        if (qn >= 64) drain_kids(64);
      }
    }
    while (sn > 0) {
      drain_slow(sn < 64 ? sn : 64);
      if (qn >= 64) drain_kids(64);
    }
    while (qn > 0) drain_kids(qn < 64 ? qn : 64);
    if (lc.dep) atomicAdd(&s_cnt[PIC_C_ALIVE], (unsigned long long)lc.dep);
    if (lc.tr) atomicAdd(&s_cnt[PIC_C_TRANSMIT], (unsigned long long)lc.tr);
    if (lc.ri) atomicAdd(&s_cnt[PIC_C_REFL_IF], (unsigned long long)lc.ri);
    if (lc.rs) atomicAdd(&s_cnt[PIC_C_REFL_SURF], (unsigned long long)lc.rs);
    __syncthreads();
    if (tid == 0) {
      int nt = tail0 + s_app;
      if (nt > cap) nt = cap;
      a.slab_tail[slab] = nt;
      a.slab_dead[slab] += s_dead;
    }
  }
  if (cur_inst >= 0) flush_bins<MODE>(a, s_inst, s_dens, s_cur);
  if (bad) atomicOr(a.status, kStHits);
  if (n_fast) atomicAdd(&s_fast, (unsigned long long)n_fast);
  if (n_left) atomicAdd(&s_left, (unsigned long long)n_left);
  __syncthreads();
  if (tid < kNC && s_cnt[tid])
    atomicAdd((unsigned long long*)&a.counters[(int64_t)a.step * kNC + tid], s_cnt[tid]);
  if (tid == 0) {
    if (s_fast) atomicAdd(&a.stats[(int64_t)a.step * 2 + 0], s_fast);
    if (s_left) atomicAdd(&a.stats[(int64_t)a.step * 2 + 1], s_left);
  }
}

// In-place compaction of slabs whose tombstones exceed a fraction of their tail.  One
// workgroup per slab walks it tile by tile: every lane loads its slot, a workgroup scan
// of the live lanes gives the destination, and the stores follow a barrier, so a
// destination (always <= its source) is never overwritten before it has been read.
template <typename F>
__global__ void __launch_bounds__(1024) k_compact(CompactArgs a) {
  __shared__ int s_w[16];
  const int slab = blockIdx.x;
  const int tail = a.slab_tail[slab];
  const int dead = a.slab_dead[slab];
  if (tail == 0 || !((float)dead > a.frac * (float)tail)) return;
  const int64_t base = a.slab_base[slab];
  const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  F* gz = (F*)a.z;
  F* gmu = (F*)a.mu;
  int out = 0;
  for (int tb = 0; tb < tail; tb += blockDim.x) {
    const int t = tb + tid;
    const bool have = t < tail;
    uint32_t fl = have ? a.flags[base + t] : kDead;
    const bool keep = !(fl & kDead);
    F z = 0, mu = 0;
    uint32_t E = 0;
    uint64_t u = 0, ev = 0;
    double row[kMaxCausalK];
    double rr = 0.0;
    if (keep) {
      z = gz[base + t];
      mu = gmu[base + t];
      E = a.E[base + t];
      u = a.uid[base + t];
      if (a.ev) ev = a.ev[base + t];
      if (a.S) {
#pragma unroll
        for (int k = 0; k < kMaxCausalK; ++k)
          if (k < a.K) row[k] = a.S[(base + t) * a.K + k];
      }
      if (a.r) rr = a.r[base + t];
    }
    const uint64_t m = __ballot(keep);
    if (lane == 0) s_w[wave] = __popcll(m);
    __syncthreads();
    int woff = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
      const int c = s_w[w];
      woff += w < wave ? c : 0;
      tot += c;
    }
    if (keep) {
      const int64_t d = base + out + woff + __popcll(m & lanes_below());
      gz[d] = z;
      gmu[d] = mu;
      a.E[d] = E;
      a.uid[d] = u;
      a.flags[d] = fl;
      if (a.ev) a.ev[d] = ev;
      if (a.S) {
#pragma unroll
        for (int k = 0; k < kMaxCausalK; ++k)
          if (k < a.K) a.S[d * a.K + k] = row[k];
      }
      if (a.r) a.r[d] = rr;
    }
    out += tot;
    __syncthreads();
  }
  if (tid == 0) {
    a.slab_tail[slab] = out;
    a.slab_dead[slab] = 0;
  }
}

__global__ void k_fill32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_convert(const uint64_t* dens, int64_t nd, const int64_t* cur, int64_t nc,
                          double* dout, double* cout) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd || i < nc;
       i += stride) {
    if (dout && i < nd) dout[i] = (double)dens[i];
    if (cout && i < nc) cout[i] = (double)cur[i] * 0x1p-32;
  }
}

template <typename F, int MODE>
static void launch_mode(const StepArgs& a, const StepLaunch& L, hipStream_t s) {
  if (L.ev[0]) (void)hipEventRecord(L.ev[0], s);
  hipLaunchKernelGGL((k_step<F, MODE>), dim3(L.grid), dim3(L.block), L.lds, s, a);
  if (L.ev[1]) (void)hipEventRecord(L.ev[1], s);
}

template <typename F>
static hipError_t launch_prec(const StepArgs& a, int mode, const StepLaunch& L, hipStream_t s) {
  switch (mode) {
#define PIC_MODE(m) \
  case m:           \
    launch_mode<F, m>(a, L, s); \
    break;
    PIC_MODE(0) PIC_MODE(1) PIC_MODE(2) PIC_MODE(3) PIC_MODE(4) PIC_MODE(5)
    PIC_MODE(8) PIC_MODE(9) PIC_MODE(10) PIC_MODE(11) PIC_MODE(12) PIC_MODE(13)
#undef PIC_MODE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t step_static_lds() {
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_step<double, kModeDensLds | kModeCur>)) != hipSuccess)
    return 8192;
  return fa.sharedSizeBytes;
}

template <typename F, int MODE>
static hipError_t raise_lds(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step<F, MODE>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t set_step_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
#define PIC_RAISE(m)                                         \
  if (e == hipSuccess) e = raise_lds<float, m>(bytes);       \
  if (e == hipSuccess) e = raise_lds<double, m>(bytes);
  PIC_RAISE(0) PIC_RAISE(1) PIC_RAISE(2) PIC_RAISE(3) PIC_RAISE(4) PIC_RAISE(5)
  PIC_RAISE(8) PIC_RAISE(9) PIC_RAISE(10) PIC_RAISE(11) PIC_RAISE(12) PIC_RAISE(13)
#undef PIC_RAISE
  return e;
}

hipError_t launch_step(const StepArgs& a, bool fp64, const StepLaunch& L, hipStream_t s) {
  const int mode = (a.debug ? kModeDebug : 0) |
                   (a.dens_on ? (a.dens_lds ? kModeDensLds : kModeDensGlobal) : 0) |
                   (a.cur_on ? kModeCur : 0);
  return fp64 ? launch_prec<double>(a, mode, L, s) : launch_prec<float>(a, mode, L, s);
}

hipError_t launch_compact(const CompactArgs& a, bool fp64, int block, hipStream_t s) {
  if (a.n_slabs <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(k_compact<double>, dim3(a.n_slabs), dim3(block), 0, s, a);
  else
    hipLaunchKernelGGL(k_compact<float>, dim3(a.n_slabs), dim3(block), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_convert(const uint64_t* dens, int64_t nd, const int64_t* cur, int64_t nc,
                          double* dout, double* cout, hipStream_t s) {
  const int64_t n = nd > nc ? nd : nc;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, s, dens, nd, cur, nc,
                     dout, cout);
  return hipGetLastError();
}

}  // namespace pic
