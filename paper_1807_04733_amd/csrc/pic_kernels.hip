// Device kernels of the hot-electron particle-in-cell step for gfx950 (CDNA4, wave64).
//
// One launch of k_step advances every carrier of every instance by one or two steps of
// the Strang splitting of arXiv:1807.04733 Eq. (15):
//   Source(dt/2)     primaries scheduled for the step are appended with their initial
//                    state (Eq. 17)
//   Transport(dt/2)  straight flight, vacuum reflection, stochastic interfaces (Eq. 18)
//   Scattering(dt)   Monte-Carlo event with p = 1 - exp(-dt/tau_eff) (Eq. 2, Sec. III.A):
//                    elastic (Eq. 8) or inelastic with an energy-conserving secondary
//                    (Eqs. 6-7, 19); products below E_min are removed (at once, or at
//                    their next event)
//   Transport(dt/2)  for the survivor and the newborn
//   deposit          density and v*cos(theta) moments (Eqs. 16, 23) into LDS histograms,
//                    optionally the generation label and superparticle weights (Eq. 10)
//
// Speeds and inelastic rates are per-channel constants or energy tables (Fig. 1); each
// option is a compile-time mode so that the plain kernel carries none of its code.
// Data layout: structure-of-arrays particle state streamed once per launch (z,
// cos(theta), energy, uid, flags), partitioned into slabs that each belong to one
// instance.  A slab is processed by one workgroup per launch, which appends newborns
// behind the slab's tail with a wave ballot + one LDS atomic per wave (no global atomics
// on the append path).
// Histograms are privatised per workgroup in LDS and merged into the int64 bins with
// global atomics only for non-zero entries.  All decisions use binary64 arithmetic in
// the order written here; the file is built with -ffp-contract=off.
#include <utility>

#include "pic_device.h"

#pragma clang fp contract(off)

namespace pic {

// Compile-time launch modes of the step kernel.
constexpr int kModeDebug = 1;       // keep per-particle event counts
constexpr int kModeDensGlobal = 4;  // density with global atomics (its LDS slice does not fit)
constexpr int kModeTab = 8;         // energy-dependent speeds and rates (tables in LDS)
constexpr int kModeWt = 16;         // weighted superparticles (StepArgs::wt)
constexpr int kModeDens16 = 32;     // density slices as 16-bit counters, two per LDS word
// The whole-tree likelihood-ratio adjoint replays the run twice with the same dynamics and
// launch structure as the forward (two steps per launch from registers where carriers stay
// on the common path).  Pass 1 deposits nothing: each deposit adds its weight in the loss,
// dL/d(density) + dL/d(current) v cos(theta), to the carrier's partial return, and the
// partial returns add up to the return R of each primary tree.  Pass 2 adds every score
// term of the tree's random decisions times R to the gradient (the non-event terms of a
// carrier lazily, from the first pending step kept in its flags).
constexpr int kModeRet = 64;        // whole-tree adjoint, pass 1
constexpr int kModeScore = 128;     // whole-tree adjoint, pass 2

// Compile-time sub-step index for the generic lambdas of k_step.
template <int V>
struct Sub {
  static constexpr int value = V;
};

// weighted moments: the density and generation slices hold u64 sums of weights
template <int MODE>
__device__ __forceinline__ bool weighted(const StepArgs& a) {
  return (MODE & kModeWt) != 0;
}

// A 16-bit density counter of the LDS slice wrapped (rare: 65536 deposits into one bin of
// one workgroup's slice).  The 32-bit word k holds bin 2k (spin up of a cell) in its low
// and bin 2k+1 (spin down) in its high half and only ever receives additions, so every
// wrap of a half is seen by exactly the atomic that causes it (from the value it returns):
// that lane moves 65536 into the int64 bin, and a carry out of the low half into the high
// half is taken back out at once (a wrap of the high half caused by the carry or by taking
// it back out is counted the same way).  The slice then holds every bin's count modulo
// 65536 and the int64 bins the rest, exactly, whatever the order of the concurrent
// additions.
__device__ __forceinline__ void dens16_wrap(unsigned long long* g, int idx, uint32_t sh,
                                            uint32_t old, uint32_t* wd) {
  atomicAdd(&g[idx], 65536ull);
  if (sh == 0) {
    const int hi_bin = idx + 1;
    if ((old >> 16) == 0xFFFFu) atomicAdd(&g[hi_bin], 65536ull);
    const uint32_t old2 = atomicAdd(wd, 0xFFFF0000u);
    if ((old2 >> 16) == 0u) atomicAdd(&g[hi_bin], (unsigned long long)(-65536ll));
  }
}

// Deposit of one carrier at the end of sub-step J into the LDS histogram slices of that
// sub-step (density per (z, E, spin), current per (z, spin)), or density to the global
// bins when its slice does not fit in LDS.  `eb` is the energy bin, `val` the current
// value (cur_fixed / cur_fixed_w), `wfx` the weight (2^-16 units) of a weighted run.
template <int MODE, int J>
__device__ __forceinline__ void deposit_v(const StepArgs& a, const DevInst& I, unsigned char* dyn,
                                          double z, int eb, uint32_t fl, long long val,
                                          uint32_t wfx, double& racc) {
  if constexpr ((MODE & kModeScore) != 0) return;  // adjoint pass 2: no moments
  int zb = (int)floor(z * I.inv_dz);
  zb = zb < 0 ? 0 : (zb > I.nz - 1 ? I.nz - 1 : zb);
  const int s = (int)(fl & kSpinMask);
  if constexpr ((MODE & kModeRet) != 0) {
    // adjoint pass 1: the deposit's weight in the loss joins the carrier's partial return
    double g = 0.0;
    if (a.sub_dens_on[J] && a.adj_gd) {
      const double gd = a.adj_gd[I.dens_off +
                                 (((int64_t)a.sub_dens_slot[J] * I.nz + zb) * a.n_ebins + eb) * 2 + s];
      g += weighted<MODE>(a) ? gd * ((double)wfx * 0x1p-16) : gd;
    }
    if (a.sub_cur_on[J] && a.adj_gc) {
      const double gc = ((const double*)(dyn + a.lds_cur_at[J]))[zb * 2 + s];
      if (gc != 0.0) g += gc * ((double)val * 0x1p-32);
    }
    if (g != 0.0) racc += g;
    return;
  }
  if (a.sub_dens_on[J]) {
    const int idx = (zb * a.n_ebins + eb) * 2 + s;
    const bool wtd = weighted<MODE>(a);
    const unsigned long long add = wtd ? (unsigned long long)wfx : 1ull;
    if (MODE & kModeDensGlobal) {
      const int64_t g = I.dens_off + (int64_t)a.sub_dens_slot[J] * I.nz * a.n_ebins * 2 + idx;
      atomicAdd((unsigned long long*)&a.dens[g], add);
    } else if (MODE & kModeDens16) {
      uint32_t* wd = (uint32_t*)(dyn + a.lds_dens_at[J]) + (idx >> 1);
      const uint32_t sh = (uint32_t)(idx & 1) << 4;
      const uint32_t old = atomicAdd(wd, 1u << sh);
      if (__builtin_expect(((old >> sh) & 0xFFFFu) == 0xFFFFu, 0))
        dens16_wrap((unsigned long long*)(a.dens + I.dens_off +
                                          (int64_t)a.sub_dens_slot[J] * I.nz * a.n_ebins * 2),
                    idx, sh, old, wd);
    } else if (wtd) {
      atomicAdd((unsigned long long*)(dyn + a.lds_dens_at[J]) + idx, add);
    } else {
      atomicAdd((uint32_t*)(dyn + a.lds_dens_at[J]) + idx, 1u);
    }
    if (a.gen) {  // generation label, summed per (z, spin)
      const uint32_t gl = (fl >> kGenShift) & kGenMask;
      if (MODE & kModeDensGlobal) {
        const int64_t g = I.gen_off + ((int64_t)a.sub_dens_slot[J] * I.nz + zb) * 2 + s;
        atomicAdd((unsigned long long*)&a.gen[g], (unsigned long long)gl * add);
      } else if (wtd) {
        atomicAdd((unsigned long long*)(dyn + a.lds_gen_at[J]) + zb * 2 + s,
                  (unsigned long long)gl * add);
      } else {
        atomicAdd((uint32_t*)(dyn + a.lds_gen_at[J]) + zb * 2 + s, gl);
      }
    }
  }
  if (a.sub_cur_on[J])
    atomicAdd((unsigned long long*)(dyn + a.lds_cur_at[J]) + zb * 2 + s, (unsigned long long)val);
}

// energy bin of E for the density deposit (0 with a single bin)
__device__ __forceinline__ int ebin(const StepArgs& a, const uint32_t* s_edges,
                                    const uint8_t* s_ebkt, uint32_t E) {
  return a.n_ebins > 1 ? energy_bin_b(s_edges, s_ebkt, a.n_ebins, E) : 0;
}

// current value of a carrier (weighted in a weighted run)
template <int MODE>
__device__ __forceinline__ long long cur_val(const StepArgs& a, double v, double mu,
                                             uint32_t wfx) {
  return weighted<MODE>(a) ? cur_fixed_w(v, mu, wfx) : cur_fixed(v, mu);
}

template <int MODE, int J>
__device__ __forceinline__ void deposit(const StepArgs& a, const DevInst& I, unsigned char* dyn,
                                        const uint32_t* s_edges, const uint8_t* s_ebkt, double z,
                                        double mu, uint32_t E, uint32_t fl, double v,
                                        uint32_t wfx, double& racc) {
  if constexpr ((MODE & kModeScore) != 0) return;
  const int eb = a.sub_dens_on[J] ? ebin(a, s_edges, s_ebkt, E) : 0;
  deposit_v<MODE, J>(a, I, dyn, z, eb, fl, cur_val<MODE>(a, v, mu, wfx), wfx, racc);
}

// Score terms of adjoint pass 2: added to the workgroup's gradient accumulator in LDS,
// times the return R of the carrier's tree.
struct TreeScore {
  double* s_grad;
  double R;
  __device__ __forceinline__ void add(int k, double v) const { atomicAdd(&s_grad[k], v * R); }
  // the pending non-event terms, +x_in for each step from the first pending one to upto-1
  // (a constant channel), folded in
  __device__ __forceinline__ void flush(uint32_t& fl, uint32_t upto, int chan, double x_in) const {
    const uint32_t nf = nf_of(fl);
    if (upto > nf) {
      add(chan, (double)(upto - nf) * x_in);
      fl = with_nf(fl, upto);
    }
  }
};

// Interface decisions of a half step in adjoint pass 2: the pending non-event terms of the
// channel before the hit, then the score of the transmission draw on the table nodes that
// the carrier's energy interpolates, w0/T and w1/T if transmitted, -w/(1-T) if reflected.
struct HitTreeScore {
  const TreeScore& ts;
  const DevInst& I;
  const double* et;
  bool tau2;
  double dt;
  uint32_t& fl;
  uint32_t E;
  uint32_t upto;
  __device__ __forceinline__ void operator()(int tab, int layer, double T, bool go) const {
    const int s = (int)(fl & kSpinMask);
    ts.flush(fl, upto, I.chi[layer][s], dt * inel_rate_at(I, et, tau2, layer, s, E));
    const int TE = I.t_entries;
    int k0 = 0;
    double w0 = 1.0, w1 = 0.0;
    if (TE > 1) {
      const double x = ((double)E * 0x1p-30) * I.T_scale;
      const int k = (int)floor(x);
      if (k >= TE - 1) {
        k0 = TE - 1;
      } else {
        k0 = k;
        w1 = x - (double)k;
        w0 = 1.0 - w1;
      }
    }
    const int base = (int)I.n_ch + tab * TE + k0;
    if (go) {
      ts.add(base, w0 / T);
      if (w1 != 0.0) ts.add(base + 1, w1 / T);
    } else {
      ts.add(base, -w0 / (1.0 - T));
      if (w1 != 0.0) ts.add(base + 1, -w1 / (1.0 - T));
    }
  }
};

// Merge one LDS histogram slice of n entries (u32 or u64) into int64 bins (non-zero
// entries only) and clear it.
template <typename U>
__device__ __forceinline__ void merge_slice(U* s, unsigned long long* g, int n) {
  for (int b = threadIdx.x; b < n; b += blockDim.x) {
    const U v = s[b];
    if (v) {
      atomicAdd(&g[b], (unsigned long long)v);
      s[b] = 0;
    }
  }
}

// The same for a slice of n 16-bit counters packed two per 32-bit word (n even; word k
// holds bins 2k and 2k+1).
__device__ __forceinline__ void merge_slice16(uint32_t* s, unsigned long long* g, int n) {
  for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
    const uint32_t v = s[b];
    if (v) {
      if (v & 0xFFFFu) atomicAdd(&g[2 * b], (unsigned long long)(v & 0xFFFFu));
      if (v >> 16) atomicAdd(&g[2 * b + 1], (unsigned long long)(v >> 16));
      s[b] = 0;
    }
  }
}

// Merge sub-step J's LDS histogram slices of the workgroup's instance into the int64 bins
// and clear them.
template <int MODE, int J>
__device__ void flush_bins(const StepArgs& a, const DevInst& I, unsigned char* dyn) {
  if (!(MODE & kModeDensGlobal) && a.sub_dens_on[J]) {
    const bool wtd = weighted<MODE>(a);
    const int n = I.nz * a.n_ebins * 2;
    unsigned long long* g =
        (unsigned long long*)(a.dens + I.dens_off + (int64_t)a.sub_dens_slot[J] * n);
    if (wtd) merge_slice((unsigned long long*)(dyn + a.lds_dens_at[J]), g, n);
    else if (MODE & kModeDens16) merge_slice16((uint32_t*)(dyn + a.lds_dens_at[J]), g, n);
    else merge_slice((uint32_t*)(dyn + a.lds_dens_at[J]), g, n);
    if (a.gen) {
      const int m = I.nz * 2;
      unsigned long long* gg =
          (unsigned long long*)(a.gen + I.gen_off + (int64_t)a.sub_dens_slot[J] * m);
      if (wtd) merge_slice((unsigned long long*)(dyn + a.lds_gen_at[J]), gg, m);
      else merge_slice((uint32_t*)(dyn + a.lds_gen_at[J]), gg, m);
    }
  }
  if (a.sub_cur_on[J]) {
    const int n = I.nz * 2;
    merge_slice((unsigned long long*)(dyn + a.lds_cur_at[J]),
                (unsigned long long*)(a.cur + I.cur_off + (int64_t)a.sub_cur_slot[J] * n), n);
  }
}

template <int MODE, int T>
__device__ void flush_all(const StepArgs& a, const DevInst& I, unsigned char* dyn) {
  __syncthreads();
  flush_bins<MODE, 0>(a, I, dyn);
  if constexpr (T > 1) flush_bins<MODE, 1>(a, I, dyn);
  __syncthreads();
}

// Newborn secondaries of one general pass wait in a wave-private LDS queue and are
// finished right after it, 64 at a time, so the spawn draw, the newborn's half step, its
// deposit and its append run as full waves instead of once per wave for a few lanes.
constexpr int kQ = 64;
struct ChildQueue {  // kChildQueueBytes
  double z[kQ];
  uint32_t lo[kQ], hi[kQ], E[kQ], fl[kQ], w[kQ];
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
  uint32_t* w;
  double* r;     // adjoint pass 1: partial returns
};

// Element i of a slab array, addressed with a 32-bit byte offset from the slab's base
// (a slab holds fewer than 2^28 slots), so that the access can use the scalar base + vector
// offset form of global memory instructions.
template <typename T>
__device__ __forceinline__ T& at(T* base, uint32_t i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}

struct LaneCounts {
  uint32_t dep, tr, ri, rs;
};

// Per-wave queues of general-path slots: sub-step 0 holds < 64 + 64 entries; sub-step 1
// also receives the survivors and newborns of a sub-step-0 general pass (< 64 + 64 + 128).
constexpr int kSlowQ0 = 128;
constexpr int kSlowQ1 = 256;
// rounds of tiles at the end of a slab handed out on demand (the rest are interleaved)
constexpr int kDynRounds = 16;

// One launch of k_step advances every carrier of every instance by T (1 or 2) steps of the
// Strang splitting.  A workgroup takes one slab at a time; each lane takes one carrier
// per iteration and runs its T steps from registers while they stay on the common path:
// no layer boundary in either half step and a scattering draw at or above x = dt/tau_eff
// (which is above p = 1 - exp(-x), so no event can happen).  The first step that leaves
// the common path puts the carrier's slot into the wave's LDS queue of that sub-step; the
// state in HBM is still the one stored before it (its z stamp says which straight
// flights to redo), and the sub-step-0 queue keeps a copy of it in LDS where that fits.
// A queue of 64 slots runs the general path as a full wave; the
// survivors and newborns of a sub-step-0 general pass continue with sub-step 1 the same
// way.  New primaries (source term, Eq. 17) of a sub-step are appended with their initial
// state and queued for its general path.
template <typename F, int T, int MODE>
__global__ void __launch_bounds__(1024, 4) k_step(StepArgs a) {
  constexpr bool DEBUG = (MODE & kModeDebug) != 0;
  constexpr bool ET = (MODE & kModeTab) != 0;
  constexpr bool RET = (MODE & kModeRet) != 0;      // adjoint pass 1
  constexpr bool SCORE = (MODE & kModeScore) != 0;  // adjoint pass 2
  constexpr bool ADJP = RET || SCORE;
  // dynamic LDS: [histogram slices of the sub-steps | energy tables | per wave: newborn
  // queue, slot queue of sub-step 0 (, of sub-step 1) | per wave, where they fit: copies of
  // the stored state of the sub-step-0 queue's carriers]; offsets set by the host
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ DevInst s_inst;
  __shared__ unsigned long long s_cnt[T][kNC];
  __shared__ uint32_t s_edges[PIC_MAX_EBINS];
  __shared__ __align__(4) uint8_t s_ebkt[kEBuckets];
  __shared__ int s_slab, s_app, s_dead, s_tile;
  __shared__ unsigned long long s_fast[T], s_left[T];

  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int wave = tid >> 6;
  for (int i = tid; i < a.lds_q_at / 4; i += blockDim.x) ((uint32_t*)dyn)[i] = 0;
  for (int i = tid; i < a.n_ebins; i += blockDim.x) s_edges[i] = a.e_edges[i];
  for (int i = tid; i < kEBuckets / 4; i += blockDim.x)
    ((uint32_t*)s_ebkt)[i] = ((const uint32_t*)a.e_bucket)[i];
  for (int i = tid; i < T * kNC; i += blockDim.x) (&s_cnt[0][0])[i] = 0;
  if (tid < T) {
    s_fast[tid] = 0;
    s_left[tid] = 0;
  }
  uint32_t n_fast[T], n_left[T];
#pragma unroll
  for (int j = 0; j < T; ++j) n_fast[j] = n_left[j] = 0;

  F* gz = (F*)a.z;
  F* gmu = (F*)a.mu;
  const uint32_t step0 = (uint32_t)a.step;
  unsigned char* wq = dyn + a.lds_q_at + (size_t)wave * a.lds_q_bytes;
  ChildQueue& Q = *(ChildQueue*)wq;
  uint32_t* const SQ0 = (uint32_t*)(wq + kChildQueueBytes);
  uint32_t* const SQ1 = SQ0 + kSlowQ0;
  // copies of the state of the carriers in SQ0, entry for entry (when staged): z, cos(theta),
  // E, flags, uid as they are stored in the particle arrays
  const bool STG = a.lds_stage_at >= 0;
  static_assert(stage_wave_bytes(sizeof(F) == 8) == kSlowQ0 * (2 * sizeof(F) + 16), "stage");
  F* const st_z = (F*)(dyn + (STG ? a.lds_stage_at : 0) +
                       (size_t)wave * stage_wave_bytes(sizeof(F) == 8));
  F* const st_mu = st_z + kSlowQ0;
  uint32_t* const st_E = (uint32_t*)(st_mu + kSlowQ0);
  uint32_t* const st_fl = st_E + kSlowQ0;
  uint64_t* const st_u = (uint64_t*)(st_fl + kSlowQ0);
  // the same for the first kStage1 entries of the sub-step-1 queue (when staged)
  const bool STG1 = T > 1 && a.lds_stage1_at >= 0;
  F* const s1_z = (F*)(dyn + (STG1 ? a.lds_stage1_at : 0) +
                       (size_t)wave * stage1_wave_bytes(sizeof(F) == 8));
  F* const s1_mu = s1_z + kStage1;
  uint32_t* const s1_E = (uint32_t*)(s1_mu + kStage1);
  uint32_t* const s1_fl = s1_E + kStage1;
  uint64_t* const s1_u = (uint64_t*)(s1_fl + kStage1);
  static_assert(sizeof(ChildQueue) == kChildQueueBytes, "queue layout");
  const double* const et = ET ? (const double*)(dyn + a.lds_etab_at) : nullptr;
  const bool tau2 = a.tau_exp2 != 0;
  const bool WT = weighted<MODE>(a);
  double* const s_grad = SCORE ? (double*)(dyn + a.lds_grad_at) : nullptr;
  constexpr uint32_t kW1 = 1u << 16;  // weight 1
  int cur_inst = -1;
  bool bad = false;

  for (;;) {
    if (tid == 0) s_slab = atomicAdd(&a.queue[a.step], 1);
    __syncthreads();
    const int slab = __builtin_amdgcn_readfirstlane(s_slab);
    if (slab >= a.n_slabs) break;
    const int inst = a.slab_inst[slab];
    if (inst != cur_inst) {
      if constexpr (ADJP) {
        if (cur_inst >= 0) __syncthreads();  // every wave is done with the old tables
      } else {
        if (cur_inst >= 0) flush_all<MODE, T>(a, s_inst, dyn);
      }
      const uint4* src = (const uint4*)&a.inst[inst];
      uint4* dst = (uint4*)&s_inst;
      for (int i = tid; i < a.inst_bytes / 16; i += blockDim.x) dst[i] = src[i];
      if constexpr (ET) {
        const DevInst& G = a.inst[inst];
        const int n = 2 * (int)G.n_ch * G.e_nodes;
        const double* tsrc = a.etab + G.etab_off;
        double* tdst = (double*)(dyn + a.lds_etab_at);
        for (int i = tid; i < n; i += blockDim.x) tdst[i] = tsrc[i];
      }
      if constexpr (RET) {
        // this instance's dL/d(current) slices of the launch's steps
        const DevInst& G = a.inst[inst];
        for (int j = 0; j < T; ++j)
          if (a.sub_cur_on[j] && a.adj_gc) {
            const double* gsrc = a.adj_gc + G.cur_off + (int64_t)a.sub_cur_slot[j] * G.nz * 2;
            double* gdst = (double*)(dyn + a.lds_cur_at[j]);
            for (int i = tid; i < G.nz * 2; i += blockDim.x) gdst[i] = gsrc[i];
          }
      }
      cur_inst = inst;
    }
    if (tid == 0) {
      s_app = 0;
      s_dead = 0;
      s_tile = 0;
    }
    __syncthreads();
    const DevInst& I = s_inst;
    const int64_t base = a.slab_base[slab];
    const int cap = a.slab_cap[slab];
    const int tail0 = a.slab_tail[slab];
    const int64_t kk = a.slab_k[slab];
    const int64_t S = I.n_slabs;
    const int64_t* cum = a.inj_cum + (int64_t)inst * (a.n_steps + 1);
    // primaries of sub-step j are the instance's primaries [cum[step0+j], cum[step0+j+1])
    // that fall in this slab (index = slab k mod S)
    const int64_t f00 = count_mod(cum[step0], kk, S);
    const int64_t f01 = count_mod(cum[step0 + 1], kk, S);
    const int n_inj0 = (int)(f01 - f00);
    int n_inj1 = 0;
    if constexpr (T > 1) n_inj1 = (int)(count_mod(cum[step0 + 2], kk, S) - f01);
    const int total = tail0 + n_inj0 + n_inj1;
    if (tid == 0) {
      if (n_inj0) atomicAdd(&s_cnt[0][PIC_C_INJECTED], (unsigned long long)n_inj0);
      if constexpr (T > 1)
        if (n_inj1) atomicAdd(&s_cnt[T - 1][PIC_C_INJECTED], (unsigned long long)n_inj1);
      if (!WT) {  // weight 1 each (weighted primaries add theirs at injection)
        if (n_inj0) atomicAdd(&s_cnt[0][PIC_C_W_INJECTED], (unsigned long long)n_inj0 << 16);
        if constexpr (T > 1)
          if (n_inj1)
            atomicAdd(&s_cnt[T - 1][PIC_C_W_INJECTED], (unsigned long long)n_inj1 << 16);
      }
    }
    const SlabPtrs<F> sp{gz + base, gmu + base, a.E + base, a.uid + base, a.flags + base,
                         DEBUG ? a.ev + base : nullptr, WT ? a.wt + base : nullptr,
                         RET ? a.adj_r + base : nullptr};
    LaneCounts lc[T];
#pragma unroll
    for (int j = 0; j < T; ++j) lc[j] = LaneCounts{0, 0, 0, 0};
    int qn = 0;   // wave-uniform fill of the newborn queue
    int sn0 = 0;  // ... of the slot queue of sub-step 0
    int sn1 = 0;  // ... of sub-step 1

    auto wave_sync = [&]() __attribute__((always_inline)) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    // ---- put the slots of the lanes with `pred` into the queue of sub-step 0 with a copy
    // of their stored state (z, cos(theta), E, flags, uid) when the queue is staged
    auto push0 = [&](bool pred, uint32_t slot, F z, F mu, uint32_t E, uint32_t fl,
                     uint64_t u) __attribute__((always_inline)) {
      const uint64_t m = __ballot(pred);
      if (m) {
        if (pred) {
          const int q = sn0 + prefix_count(m);
          SQ0[q] = slot;
          if (STG) {
            st_z[q] = z;
            st_mu[q] = mu;
            st_E[q] = E;
            st_fl[q] = fl;
            st_u[q] = u;
          }
          n_left[0] += 1;
        }
        sn0 += __popcll(m);
      }
    };
    // ---- put the slots of the lanes with `pred` into the queue of sub-step J >= 1, with a
    // copy of their stored state (z, cos(theta), E, flags, uid) for the first entries when
    // those are staged
    auto push = [&](auto sub, bool pred, uint32_t slot, F z, F mu, uint32_t E, uint32_t fl,
                    uint64_t u) __attribute__((always_inline)) {
      constexpr int J = decltype(sub)::value;
      static_assert(J > 0, "sub-step 0 entries go through push0");
      const uint64_t m = __ballot(pred);
      if (m) {
        if (pred) {
          const int q = sn1 + prefix_count(m);
          SQ1[q] = slot;
          if (STG1 && q < kStage1) {
            s1_z[q] = z;
            s1_mu[q] = mu;
            s1_E[q] = E;
            s1_fl[q] = fl;
            s1_u[q] = u;
          }
          n_left[J] += 1;
        }
        sn1 += __popcll(m);
      }
    };

    // ---- the common step of sub-step J from a position at its start (no replay
    // needed), or the slot goes to the sub-step's queue.  `slot` holds the carrier whose
    // stored z is that position (stamp = this sub-step's phase).
    auto cont = [&](auto sub, bool act, uint32_t slot, double z, double mu, uint32_t E,
                    uint32_t fl, uint32_t lo, uint32_t hi, uint32_t wfx, double racc)
                    __attribute__((always_inline)) {
      constexpr int J = decltype(sub)::value;
      bool left = false;
      if (act) {
        const double r_in = racc;
        const int l = layer_of(fl);
        const LayCache c = load_lay<ET>(I, et, tau2, l, (int)(fl & kSpinMask), E);
        const double zm = z + (c.v * mu) * a.h;
        const uint32_t wd = decide_word(lo, hi, step0 + J, a.key0, a.key1);
        const double x = a.dt * (inel_rate<ET>(c, tau2, E) + I.lay[l].z);
        const double ze = zm + (c.v * mu) * a.h;
        // the start lies in the layer and both half steps move the same way
        left = u01(wd) < x || ze > c.zhi || ze < c.zlo;
        if (!left) {
          const double zs = to_store<F>(ze);
          deposit<MODE, J>(a, I, dyn, s_edges, s_ebkt, zs, mu, E, fl, c.v, wfx, racc);
          lc[J].dep += 1;
          n_fast[J] += 1;
          if (a.sub_z_write[J]) {
            at(sp.z, slot) = (F)zs;
            if ((fl >> kStampShift) & kStampMask) at(sp.fl, slot) = fl & ~(kStampMask << kStampShift);
          }
          if (RET && racc != r_in) at(sp.r, slot) = racc;
        }
      }
      push(sub, left, slot, (F)z, (F)mu, E, fl, ((uint64_t)hi << 32) | lo);
    };

    // ---------------------------------------------------------------- general path
    // The whole of sub-step J for one carrier: boundary hits, the exact scattering
    // decision, elastic / inelastic events, absorption, the newborn's queueing, the append
    // of a new primary and the write-back.  All lanes of the wave call it together; lanes
    // with nothing to do pass a dead carrier.  Returns whether the carrier is alive after
    // the step, with its state and its slot.
    auto general = [&](auto sub, bool from_soa, bool is_new, uint32_t gi, double& z, double& mu,
                       uint32_t& E, uint32_t& fl, uint32_t lo, uint32_t hi, uint64_t evp,
                       uint32_t wfx, uint32_t& slot, double& racc) __attribute__((always_inline))
                       -> bool {
      constexpr int J = decltype(sub)::value;
      const uint32_t step = step0 + J;
      // stamp of the z this sub-step stores (0 when it ends a write-back period)
      const uint32_t z_next = a.sub_z_write[J] ? 0u : (uint32_t)a.sub_z_phase[J] + 1u;
      const bool alive0 = !(fl & kDead);
      bool died = false, spawn = false;
      uint32_t dirty = 0;  // 1: mu, 2: E, 4: flags
      double zmid = 0.0;
      uint32_t E2 = 0, flmid = 0;
      HitCounts hc{0, 0, 0};
      // adjoint pass 2: the tree's return, loaded before the half step so that its latency
      // overlaps the transport arithmetic
      TreeScore ts{s_grad, 0.0};
      if (SCORE && alive0) ts.R = a.adj_R[lo];
      if (alive0) {
        const double mu_in = mu;
        const uint32_t fl_in = fl;
        LayCache c = load_lay<ET>(I, et, tau2, layer_of(fl), (int)(fl & kSpinMask), E);
        if constexpr (SCORE) {
          const uint32_t E_now = E;
          half_push_c<ET>(I, et, tau2, c, z, mu, fl, E, lo, hi, step, kTagHalf1, a.h, a.key0,
                          a.key1, hc, bad, HitTreeScore{ts, I, et, tau2, a.dt, fl, E_now, step});
        } else {
          half_push_c<ET>(I, et, tau2, c, z, mu, fl, E, lo, hi, step, kTagHalf1, a.h, a.key0,
                          a.key1, hc, bad);
        }
        // ---- scattering over the full step, at the mid-step state
        const double itel = I.lay[layer_of(fl)].z;
        const double rate = inel_rate<ET>(c, tau2, E) + itel;
        const double x = a.dt * rate;
        const double u0 = u01(decide_word(lo, hi, step, a.key0, a.key1));
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
        // the event's own words: channel (y), new direction (z), energy split (w)
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (event) w = philox10(lo, hi, step, kTagScat, a.key0, a.key1);
        if (SCORE && event) {
          // the event's score (Eq. 2), after the channel's pending non-event terms, and the
          // channel choice's (Eqs. 5, 8); non-event terms pend again from the next step
          const int cch = I.chi[layer_of(fl)][fl & kSpinMask];
          const double x_in = a.dt * inel_rate<ET>(c, tau2, E);
          ts.flush(fl, step, cch, x_in);
          const double prob = -expm1(-x);
          ts.add(cch, -x_in * exp(-x) / prob);
          const bool removed = a.absorb_next && E < a.e_min;
          if (itel > 0.0 && !removed)
            ts.add(cch, u01(w.y) < itel / rate ? x_in / x : -1.0 + x_in / x);
          fl = with_nf(fl, step + 1);
        }
        if (event && a.absorb_next && E < a.e_min) {
          // a carrier of the lowest energy bin leaves the population at its next event
          if (DEBUG) evp += 1ull;
          died = true;
          atomicAdd(&s_cnt[J][PIC_C_ABSORBED], 1ull);
          atomicAdd(&s_cnt[J][PIC_C_E_ABSORBED], (unsigned long long)E);
        } else if (event) {
          if (DEBUG) evp += 1ull;
          const bool elastic = itel > 0.0 && u01(w.y) < itel / rate;
          mu = to_store<F>(dircos(w.z));
          dirty |= 1u;
          if (elastic) {
            atomicAdd(&s_cnt[J][PIC_C_EV_EL], 1ull);
          } else {
            atomicAdd(&s_cnt[J][PIC_C_EV_EE], 1ull);
            const uint32_t E1 = __umulhi(w.w, E);
            E2 = E - E1;
            E = E1;
            dirty |= 2u;
            if (a.secondaries) {
              // with removal at the next event every secondary is created
              if (E2 >= a.e_min || a.absorb_next) {
                spawn = true;
                zmid = z;
                flmid = fl;
                if (DEBUG) evp += 1ull << 48;
                atomicAdd(&s_cnt[J][PIC_C_SPAWNED], 1ull);
              } else {
                atomicAdd(&s_cnt[J][PIC_C_SEC_ABSORBED], 1ull);
                atomicAdd(&s_cnt[J][PIC_C_E_ABSORBED], (unsigned long long)E2);
              }
            }
            if (E1 < a.e_min && !a.absorb_next) {
              died = true;
              atomicAdd(&s_cnt[J][PIC_C_ABSORBED], 1ull);
              atomicAdd(&s_cnt[J][PIC_C_E_ABSORBED], (unsigned long long)E1);
            }
          }
        }
        if (!died) {
          // with energy tables the speed and rate follow the new energy
          if constexpr (ET)
            if (dirty & 2u) c = load_lay<ET>(I, et, tau2, layer_of(fl), (int)(fl & kSpinMask), E);
          if constexpr (SCORE) {
            const uint32_t E_now = E;
            half_push_c<ET>(I, et, tau2, c, z, mu, fl, E, lo, hi, step, kTagHalf2, a.h, a.key0,
                            a.key1, hc, bad,
                            HitTreeScore{ts, I, et, tau2, a.dt, fl, E_now, step + 1});
          } else {
            half_push_c<ET>(I, et, tau2, c, z, mu, fl, E, lo, hi, step, kTagHalf2, a.h, a.key0,
                            a.key1, hc, bad);
          }
          z = to_store<F>(z);
          deposit<MODE, J>(a, I, dyn, s_edges, s_ebkt, z, mu, E, fl, c.v, wfx, racc);
          lc[J].dep += 1;
        } else {
          z = to_store<F>(z);
          fl |= kDead;
          // adjoint pass 1: the partial return goes to the tree's return
          if (RET && racc != 0.0) atomicAdd(&a.adj_R[lo], racc);
        }
        // z is stored below: the stamp says at which step of the write-back period
        fl = (fl & ~(kStampMask << kStampShift)) | (died ? 0u : z_next << kStampShift);
        if (mu != mu_in) dirty |= 1u;
        if (fl != fl_in) dirty |= 4u;
        if (DEBUG) evp += ((uint64_t)hc.tr << 16) + ((uint64_t)(hc.ri + hc.rs) << 32);
      }
      lc[J].tr += hc.tr;
      lc[J].ri += hc.ri;
      lc[J].rs += hc.rs;

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
          Q.w[p] = wfx;  // a secondary carries its parent's weight
        }
        qn += __popcll(mq);
      }
      slot = gi;
      bool placed = from_soa;
      // ---- append the new primary (always, so that an absorbed one leaves its record)
      const uint64_t ma = __ballot(is_new);
      if (ma) {
        int off = 0;
        const int leader = __ffsll((unsigned long long)ma) - 1;
        if (lane == leader) off = atomicAdd(&s_app, __popcll(ma));
        off = __shfl(off, leader);
        if (is_new) {
          const uint32_t pos = (uint32_t)(tail0 + off + prefix_count(ma));
          slot = pos;
          if ((int)pos < cap) {
            placed = true;
            at(sp.z, pos) = (F)z;
            at(sp.mu, pos) = (F)mu;
            at(sp.E, pos) = E;
            at(sp.uid, pos) = (uint64_t)lo | ((uint64_t)hi << 32);
            at(sp.fl, pos) = fl;
            if (WT) at(sp.w, pos) = wfx;
            if (DEBUG) at(sp.ev, pos) = evp;
          } else {
            atomicOr(a.status, kStOverflow);
          }
        }
      }
      if (from_soa && alive0) {
        at(sp.z, gi) = (F)z;
        if (dirty & 1u) at(sp.mu, gi) = (F)mu;
        if (dirty & 2u) at(sp.E, gi) = E;
        if (dirty & 4u) at(sp.fl, gi) = fl;
        if (DEBUG) at(sp.ev, gi) = evp;
        if (RET && !died) at(sp.r, gi) = racc;
      }
      // the slab's dead count: carriers that died in a slot of the slab (a new primary that
      // found no free slot is not one), so that tail - dead is the live count
      const uint64_t md = __ballot(died && placed);
      if (md && lane == __ffsll((unsigned long long)md) - 1) atomicAdd(&s_dead, __popcll(md));
      return alive0 && !died && placed;
    };

    // ---- finish the newborns of the last general pass of sub-step J (at most 64): spawn
    // draw (direction, spin from the layer's equilibrium polarisation, lineage), second
    // half step, deposit, append; with a further sub-step they continue with it
    auto drain_kids = [&](auto sub) __attribute__((always_inline)) {
      constexpr int J = decltype(sub)::value;
      wave_sync();
      const int n = qn;
      qn = 0;
      if (n == 0) return;
      const uint32_t step = step0 + J;
      const uint32_t z_next = a.sub_z_write[J] ? 0u : (uint32_t)a.sub_z_phase[J] + 1u;
      const bool act = lane < n;
      const int idx = act ? lane : 0;
      double cz = Q.z[idx];
      const uint32_t lo = Q.lo[idx], phi = Q.hi[idx], cE = Q.E[idx], pfl = Q.fl[idx];
      const uint32_t cw = WT ? Q.w[idx] : kW1;
      wave_sync();
      double cmu = 0.0;
      uint32_t cfl = kDead, lin = 0, pos = 0;
      bool placed = false;
      double cr = 0.0;  // adjoint pass 1: the newborn's own partial return
      if (act) {
        const uint4 sw = philox10(lo, phi, step, kTagSpawn, a.key0, a.key1);
        const int l = layer_of(pfl);
        cmu = to_store<F>(dircos(sw.x));
        const uint32_t cs = u01(sw.y) < I.lay[l].w ? 0u : 1u;
        lin = sw.z;
        if (lin == 0u || lin == phi) {
          lin = sw.w | 1u;
          if (lin == phi) lin ^= 2u;
        }
        cfl = cs | (pfl & ~kSpinMask) | (z_next << kStampShift);
        // adjoint pass 2: a newborn's non-event terms start with the next step
        if (SCORE) cfl = with_nf(cfl, step + 1);
        HitCounts h{0, 0, 0};
        LayCache cc = load_lay<ET>(I, et, tau2, l, (int)cs, cE);
        if constexpr (SCORE) {
          const TreeScore cts{s_grad, a.adj_R[lo]};
          half_push_c<ET>(I, et, tau2, cc, cz, cmu, cfl, cE, lo, lin, step, kTagHalf2, a.h,
                          a.key0, a.key1, h, bad,
                          HitTreeScore{cts, I, et, tau2, a.dt, cfl, cE, step + 1});
        } else {
          half_push_c<ET>(I, et, tau2, cc, cz, cmu, cfl, cE, lo, lin, step, kTagHalf2, a.h,
                          a.key0, a.key1, h, bad);
        }
        cz = to_store<F>(cz);
        deposit<MODE, J>(a, I, dyn, s_edges, s_ebkt, cz, cmu, cE, cfl, cc.v, cw, cr);
        lc[J].dep += 1;
        lc[J].tr += h.tr;
        lc[J].ri += h.ri;
        lc[J].rs += h.rs;
        const uint64_t m = __ballot(1);
        int off = 0;
        const int leader = __ffsll((unsigned long long)m) - 1;
        if (lane == leader) off = atomicAdd(&s_app, __popcll(m));
        off = __shfl(off, leader);
        pos = (uint32_t)(tail0 + off + prefix_count(m));
        if ((int)pos < cap) {
          placed = true;
          at(sp.z, pos) = (F)cz;
          at(sp.mu, pos) = (F)cmu;
          at(sp.E, pos) = cE;
          at(sp.uid, pos) = (uint64_t)lo | ((uint64_t)lin << 32);
          at(sp.fl, pos) = cfl;
          if (WT) at(sp.w, pos) = cw;
          if (DEBUG) at(sp.ev, pos) = ((uint64_t)h.tr << 16) + ((uint64_t)(h.ri + h.rs) << 32);
          if (RET) at(sp.r, pos) = cr;
        } else {
          atomicOr(a.status, kStOverflow);
        }
      }
      if constexpr (J + 1 < T) cont(Sub<J + 1>{}, placed, pos, cz, cmu, cE, cfl, lo, lin, cw, cr);
    };

    // re-read the top n slots of a sub-step's queue and bring z to the start of that step
    // Pop the top n entries of the queue of sub-step Q (0 or 1) with their stored state:
    // from the queue's LDS copies where they are staged (every entry of the sub-step-0
    // queue, the first kStage1 of the sub-step-1 queue), else from the particle arrays.
    auto pop_state = [&](auto which, uint32_t* SQ, int& sn, int n, int phase, bool staged,
                         uint32_t& g, double& z, double& mu, uint32_t& E, uint32_t& fl,
                         uint32_t& lo, uint32_t& hi, uint64_t& evp, uint32_t& wfx,
                         double& racc) __attribute__((always_inline)) -> bool {
      constexpr int Q = decltype(which)::value;
      wave_sync();
      const bool act = lane < n;
      const int q = sn - n + lane;
      g = act ? SQ[q] : 0u;
      // the queue entries (and their staged copies) are read before any later push
      // reuses them
      F sz = 0, smu = 0;
      uint32_t sE = 0, sfl = kDead;
      uint64_t su = 0;
      const bool stg = staged && act && (Q == 0 || q < kStage1);
      if (stg) {
        sz = Q == 0 ? st_z[q] : s1_z[q];
        smu = Q == 0 ? st_mu[q] : s1_mu[q];
        sE = Q == 0 ? st_E[q] : s1_E[q];
        sfl = Q == 0 ? st_fl[q] : s1_fl[q];
        su = Q == 0 ? st_u[q] : s1_u[q];
      }
      sn -= n;
      wave_sync();
      fl = kDead;
      if (act) {
        uint64_t u;
        if (stg) {
          fl = sfl;
          z = (double)sz;
          mu = (double)smu;
          E = sE;
          u = su;
        } else {
          fl = at(sp.fl, g);
          z = (double)at(sp.z, g);
          mu = (double)at(sp.mu, g);
          E = at(sp.E, g);
          u = at(sp.uid, g);
        }
        lo = (uint32_t)u;
        hi = (uint32_t)(u >> 32);
        if (DEBUG) evp = at(sp.ev, g);
        wfx = WT ? at(sp.w, g) : kW1;
        if (RET) racc = at(sp.r, g);
        const int d = phase - (int)((fl >> kStampShift) & kStampMask);
        if (d > 0) {
          const double v = ET ? speed_at(I, et, layer_of(fl), (int)(fl & kSpinMask), E)
                              : I.chan[layer_of(fl)][fl & kSpinMask].x;
          z = replay_flights<F>(z, (v * mu) * a.h, d);
        }
      }
      return act;
    };
    // ---- the last sub-step of the launch through the general path, for the top n slots
    // of its queue
    auto drain_last = [&](int n) __attribute__((always_inline)) {
      uint32_t g = 0, E = 0, fl = kDead, lo = 0, hi = 0, slot = 0, wfx = kW1;
      double z = 0.0, mu = 0.0, racc = 0.0;
      uint64_t evp = 0;
      const bool act = pop_state(Sub<T - 1>{}, T > 1 ? SQ1 : SQ0, T > 1 ? sn1 : sn0, n,
                                 a.sub_z_phase[T - 1], T > 1 ? STG1 : STG, g, z, mu, E, fl, lo,
                                 hi, evp, wfx, racc);
      general(Sub<T - 1>{}, act, false, g, z, mu, E, fl, lo, hi, evp, wfx, slot, racc);
      drain_kids(Sub<T - 1>{});
    };
    // ---- sub-step 0 of a two-step launch through the general path for the top n slots
    // of its queue; survivors and newborns continue with sub-step 1
    auto drain_first = [&](int n) __attribute__((always_inline)) {
      if constexpr (T > 1) {
        uint32_t g = 0, E = 0, fl = kDead, lo = 0, hi = 0, slot = 0, wfx = kW1;
        double z = 0.0, mu = 0.0, racc = 0.0;
        uint64_t evp = 0;
        const bool act = pop_state(Sub<0>{}, SQ0, sn0, n, a.sub_z_phase[0], STG, g, z, mu, E,
                                   fl, lo, hi, evp, wfx, racc);
        const bool surv =
            general(Sub<0>{}, act, false, g, z, mu, E, fl, lo, hi, evp, wfx, slot, racc);
        cont(Sub<1>{}, surv, slot, z, mu, E, fl, lo, hi, wfx, racc);
        drain_kids(Sub<0>{});
      }
    };
    // ---- a new primary of sub-step J (source term, Eq. 17), the k-th of the slab's
    // share: its initial state is appended (so that even an absorbed one leaves its record)
    // with the stamp of the start of its step, and its slot queued for the general path
    auto inject = [&](auto sub, bool want, int64_t f0, int k) __attribute__((always_inline)) {
      constexpr int J = decltype(sub)::value;
      const uint64_t m = __ballot(want);
      if (!m) return;
      int off = 0;
      const int leader = __ffsll((unsigned long long)m) - 1;
      if (lane == leader) off = atomicAdd(&s_app, __popcll(m));
      off = __shfl(off, leader);
      bool placed = false;
      uint32_t pos = 0;
      F qz = 0, qmu = 0;  // the stored state, for the staged sub-step-0 queue
      uint32_t qE = 0, qfl = 0;
      uint64_t qu = 0;
      if (want) {
        pos = (uint32_t)(tail0 + off + prefix_count(m));
        const int64_t j = kk + S * (f0 + k);
        const uint32_t root = (uint32_t)(I.root_offset + (uint64_t)j);
        const uint4 w = philox10(root, 0u, 0xFFFFFFFFu, kTagInject, a.key0, a.key1);
        double z0;
        if (I.src_lambda > 0.0)
          z0 = I.src_lo - I.src_lambda * log1p(-u01(w.x) * I.src_cd);
        else
          z0 = I.src_lo + u01(w.x) * (I.src_hi - I.src_lo);
        const double z = to_store<F>(z0);
        const double mu = to_store<F>(dircos(w.y));
        const uint32_t s = u01(w.z) < I.src_up ? 0u : 1u;
        const uint32_t E = I.e_lo[s] + __umulhi(w.w, I.e_span[s]);
        int l = 0;
        for (int q = 1; q < I.n_layers; ++q)
          if (I.lay[q].x <= z) l = q;
        uint32_t fl = s | ((uint32_t)l << kLayerShift) | (1u << kGenShift) |
                      ((uint32_t)a.sub_z_phase[J] << kStampShift);
        // adjoint pass 2: a primary's non-event terms start with its first step
        if (SCORE) fl = with_nf(fl, step0 + J);
        if (WT) {
          // weight of the primary (Eq. 10), from the weight rows behind the energy tables
          const uint32_t wfx = primary_weight(
              I, a.etab + I.etab_off + 2 * (int)I.n_ch * I.e_nodes, (int)s, E);
          if ((int)pos < cap) at(sp.w, pos) = wfx;
          atomicAdd(&s_cnt[J][PIC_C_W_INJECTED], (unsigned long long)wfx);
        }
        if ((int)pos < cap) {
          placed = true;
          qz = (F)z;
          qmu = (F)mu;
          qE = E;
          qfl = fl;
          qu = (uint64_t)root;
          at(sp.z, pos) = qz;
          at(sp.mu, pos) = qmu;
          at(sp.E, pos) = qE;
          at(sp.uid, pos) = qu;
          at(sp.fl, pos) = qfl;
          if (DEBUG) at(sp.ev, pos) = 0;
          if (RET) at(sp.r, pos) = 0.0;
        } else {
          atomicOr(a.status, kStOverflow);
        }
      }
      if constexpr (J == 0)
        push0(placed, pos, qz, qmu, qE, qfl, qu);
      else
        push(sub, placed, pos, qz, qmu, qE, qfl, qu);
    };

    // The slot a lane will handle in its next iteration is fetched one iteration ahead,
    // unconditionally (a dead slot's fields are loaded too), so that no load waits on
    // another and each wave keeps two carriers' worth of loads in flight.
    F nz = 0, nmu = 0;
    uint32_t nE = 0, nfl = kDead;
    uint64_t nu = 0;
    double nr = 0.0;  // adjoint pass 1: the slot's partial return (only its carrier changes it)
    auto fetch = [&](int t) __attribute__((always_inline)) {
      if (t < tail0) {
        const uint32_t g = (uint32_t)t;
        nfl = at(sp.fl, g);
        nz = at(sp.z, g);
        nmu = at(sp.mu, g);
        nE = at(sp.E, g);
        nu = at(sp.uid, g);
        // adjoint pass 1: the partial returns are read and written once per launch, with
        // the non-temporal hint, so that they pass through the caches without displacing
        // what is re-read (with plain accesses the pass takes about 4 % longer)
        if (RET) nr = __builtin_nontemporal_load(&at(sp.r, g));
      } else {
        nfl = kDead;
      }
    };
    // Tiles of 64 slots: wave w streams tiles w, w + W, w + 2W, ... (W waves) up to the
    // last kDynRounds rounds of the slab, whose tiles the waves then take in turn from a
    // workgroup counter, so that a wave slowed down by general passes streams fewer of
    // them and the waves reach the end of the slab together.
    const int stat_end = total > kDynRounds * (int)blockDim.x
                             ? (total / (int)blockDim.x - kDynRounds) * (int)blockDim.x
                             : 0;
    auto next_tile = [&](int cur) __attribute__((always_inline)) -> int {
      if (cur + (int)blockDim.x < stat_end) return cur + (int)blockDim.x;
      int v = 0;
      if (lane == 0) v = stat_end + atomicAdd(&s_tile, 64);
      return __builtin_amdgcn_readfirstlane(v);
    };
    int tb = wave * 64 < stat_end ? wave * 64 : next_tile(stat_end);
    fetch(tb + lane);
    // Each iteration streams 64 slots (each lane adds at most one entry to one queue),
    // then runs the general path on full queues; past the end it empties the queues.  The
    // sub-step-1 queue then holds < 64 + 64 + 128 entries.
    for (;;) {
      const bool streaming = tb < total;
      if (!streaming && sn0 == 0 && sn1 == 0) break;
      int tb_next = tb;
      if (streaming) {
        const int t = tb + lane;
        const F rz = nz, rmu = nmu;
        const uint32_t rE = nE, rfl = nfl;
        const uint64_t ru = nu;
        const double rr = nr;
        tb_next = next_tile(tb);
        fetch(tb_next + lane);
        // the weight is read for the current tile only (not prefetched): one register less
        // held across the iteration
        const uint32_t rw = WT && t < tail0 ? at(sp.w, (uint32_t)t) : kW1;
        const bool have = t < total;
        const bool from_soa = have && t < tail0;
        const bool is_new0 = have && !from_soa && t < tail0 + n_inj0;
        const bool is_new1 = have && t >= tail0 + n_inj0;
        const uint32_t gi = (uint32_t)t;

        // ---- the common steps of this launch, from registers
        int left_at = -1;
        double racc = rr;
        if (from_soa && !(rfl & kDead)) {
          const int l = layer_of(rfl), s = (int)(rfl & kSpinMask);
          const LayCache c = load_lay<ET>(I, et, tau2, l, s, rE);
          const double mu = (double)rmu;
          const double vmh = (c.v * mu) * a.h;
          const uint32_t st = (rfl >> kStampShift) & kStampMask;
          double z = replay_flights<F>((double)rz, vmh, a.sub_z_phase[0] - (int)st);
          const double x = a.dt * (inel_rate<ET>(c, tau2, rE) + I.lay[l].z);
          // u01(w) < x  <=>  w + 0.5 < x 2^32  <=>  w < x 2^32 - 0.5 (both sides exact)
          const double thr = x * 0x1p32 - 0.5;
          const long long cv = cur_val<MODE>(a, c.v, mu, rw);
          // energy bin once for both sub-steps (E does not change on the common path)
          const int eb = (a.sub_dens_on[0] || a.sub_dens_on[T - 1]) ? ebin(a, s_edges, s_ebkt, rE) : 0;
          // the decision words of the launch's steps: one generator call per step pair
          const uint4 wp = decide_pair((uint32_t)ru, (uint32_t)(ru >> 32), step0, a.key0, a.key1);
#pragma unroll
          for (int j = 0; j < T; ++j) {
            if (left_at < 0) {
              const double zm = z + vmh;
              const uint32_t sj = step0 + (uint32_t)j;
              uint32_t wd;
              if (j == 0)
                wd = (sj & 1u) ? wp.y : wp.x;
              else if ((sj & 1u) != 0u)
                wd = wp.y;  // same pair as step0 (step0 even)
              else
                wd = decide_pair((uint32_t)ru, (uint32_t)(ru >> 32), sj, a.key0, a.key1).x;
              const double ze = zm + vmh;
              // z lies in [zlo, zhi] and both half steps move it the same way, so the
              // step stays in the layer iff its end does
              if ((double)wd < thr || ze > c.zhi || ze < c.zlo) {
                left_at = j;
              } else {
                z = to_store<F>(ze);
                if (j == 0) deposit_v<MODE, 0>(a, I, dyn, z, eb, rfl, cv, rw, racc);
                if constexpr (T > 1)
                  if (j == 1) deposit_v<MODE, T - 1>(a, I, dyn, z, eb, rfl, cv, rw, racc);
                lc[j].dep += 1;
                n_fast[j] += 1;
              }
            }
          }
          if (left_at < 0 && a.sub_z_write[T - 1]) {
            at(sp.z, gi) = (F)z;
            if (st) at(sp.fl, gi) = rfl & ~(kStampMask << kStampShift);
          }
          // adjoint pass 1: the return of the common steps, stored before a general pass
          // of sub-step 1 re-reads it
          if (RET && left_at != 0 && racc != rr) __builtin_nontemporal_store(racc, &at(sp.r, gi));
        }
        push0(left_at == 0, gi, rz, rmu, rE, rfl, ru);
        if constexpr (T > 1) push(Sub<1>{}, left_at == 1, gi, rz, rmu, rE, rfl, ru);
        // ---- new primaries of each sub-step
        inject(Sub<0>{}, is_new0, f00, t - tail0);
        if constexpr (T > 1) inject(Sub<1>{}, is_new1, f01, t - tail0 - n_inj0);
      }
      const int need = streaming ? 64 : 1;
      if (sn0 >= need) {
        if constexpr (T > 1)
          drain_first(sn0 < 64 ? sn0 : 64);
        else
          drain_last(sn0 < 64 ? sn0 : 64);
      }
      if constexpr (T > 1)
        while (sn1 >= need) drain_last(sn1 < 64 ? sn1 : 64);
      tb = tb_next;
    }
#pragma unroll
    for (int j = 0; j < T; ++j) {
      if (lc[j].dep) atomicAdd(&s_cnt[j][PIC_C_ALIVE], (unsigned long long)lc[j].dep);
      if (lc[j].tr) atomicAdd(&s_cnt[j][PIC_C_TRANSMIT], (unsigned long long)lc[j].tr);
      if (lc[j].ri) atomicAdd(&s_cnt[j][PIC_C_REFL_IF], (unsigned long long)lc[j].ri);
      if (lc[j].rs) atomicAdd(&s_cnt[j][PIC_C_REFL_SURF], (unsigned long long)lc[j].rs);
    }
    __syncthreads();
    if (tid == 0) {
      int nt = tail0 + s_app;
      if (nt > cap) nt = cap;
      a.slab_tail[slab] = nt;
      a.slab_dead[slab] += s_dead;
    }
  }
  if constexpr (!ADJP)
    if (cur_inst >= 0) flush_all<MODE, T>(a, s_inst, dyn);
  if (bad) atomicOr(a.status, kStHits);
  if constexpr (ADJP) {
    // the replays leave the forward's counters alone; pass 2 hands in its gradient
    if constexpr (SCORE) {
      __syncthreads();
      for (int k = tid; k < a.adj_K; k += blockDim.x)
        if (s_grad[k] != 0.0) atomicAdd(&a.adj_grad[k], s_grad[k]);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < T; ++j) {
    if (n_fast[j]) atomicAdd(&s_fast[j], (unsigned long long)n_fast[j]);
    if (n_left[j]) atomicAdd(&s_left[j], (unsigned long long)n_left[j]);
  }
  __syncthreads();
  for (int i = tid; i < T * kNC; i += blockDim.x) {
    const unsigned long long v = (&s_cnt[0][0])[i];
    if (v) atomicAdd((unsigned long long*)&a.counters[(int64_t)a.step * kNC + i], v);
  }
  if (tid < T) {
    if (s_fast[tid]) atomicAdd(&a.stats[((int64_t)a.step + tid) * 2 + 0], s_fast[tid]);
    if (s_left[tid]) atomicAdd(&a.stats[((int64_t)a.step + tid) * 2 + 1], s_left[tid]);
  }
}

// In-place compaction of slabs whose tombstones exceed a fraction of their tail.  With L
// live carriers in a slab, the live carriers at or above slot L move into the dead slots
// below L and the tail becomes L, so about as many carriers move as there are tombstones
// below L (the order of carriers in a slab changes no result).  L is the tail minus the
// slab's dead count, which the step kernels keep exact.  One workgroup per slab collects
// dead slots below L and live slots at or above L into two LDS rings, kScanTile slots per
// scan round, and moves them in pairs.  Sources and destinations lie on either side of L,
// so the moves need no ordering among themselves; the two counts are equal, so every dead
// slot below L is filled.  The widest workgroup does it fastest: 1024 threads with two
// slots each per round took 21.6 ms per batched run and 5.3 ms per spin-valve run against
// 23.6 and 6.2 ms with 256 threads and four slots each.
constexpr int kCompactBlock = 1024;
constexpr int kCompactPer = 2;                                // slots per thread per round
constexpr int kScanTile = kCompactBlock * kCompactPer;
constexpr int kHoleBatch = 1024;                              // dead slots per move batch
constexpr int kRingH = 4096;                                  // > kHoleBatch - 1 + kScanTile
constexpr int kRingT = 8192;                                  // > kRingH - 1 + kScanTile
static_assert(kHoleBatch - 1 + kScanTile <= kRingH && kRingH - 1 + kScanTile <= kRingT,
              "ring bounds");

template <typename F>
__global__ void __launch_bounds__(kCompactBlock) k_compact(CompactArgs a) {
  __shared__ int sH[kRingH], sT[kRingT];
  __shared__ int s_cnt[2];  // appended dead slots, appended live slots
  const int slab = blockIdx.x;
  const int tail = a.slab_tail[slab];
  const int dead = a.slab_dead[slab];
  if (tail == 0 || !((float)dead > a.frac * (float)tail)) return;
  const int64_t base = a.slab_base[slab];
  const uint32_t* const fl = a.flags + base;
  const int tid = threadIdx.x, lane = __lane_id();
  if (dead > tail) return;  // never happens: the step kernels count only dead slots
  if (tid < 2) s_cnt[tid] = 0;
  __syncthreads();
  const int L = tail - dead;
  // wave-aggregated append of slot t to a ring (absolute positions; index = position & mask)
  auto append = [&](bool want, int t, int* ring, int mask, int* ctr) {
    const uint64_t m = __ballot(want);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int off = 0;
    if (lane == leader) off = atomicAdd(ctr, __popcll(m));
    off = __shfl(off, leader);
    if (want) ring[(off + __popcll(m & lanes_below())) & mask] = t;
  };
  // one scan round over [from, from + kScanTile) ∩ [lo, hi): appends the slots whose dead
  // bit equals `want_dead`; returns the ring's new end (the same in every thread)
  auto scan = [&](int from, int hi, bool want_dead, int* ring, int mask, int* ctr) -> int {
    uint32_t f[kCompactPer];
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
      const int t = from + j * kCompactBlock + tid;
      f[j] = t < hi ? fl[t] : (want_dead ? 0u : kDead);
    }
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j)
      append(((f[j] & kDead) != 0) == want_dead, from + j * kCompactBlock + tid, ring, mask, ctr);
    __syncthreads();
    const int end = *ctr;
    __syncthreads();  // every thread has read the count before the next round appends
    return end;
  };
  F* gz = (F*)a.z;
  F* gmu = (F*)a.mu;
  int hp = 0, tp = L;    // next slot to scan below L / at or above L
  int hh = 0, ht = 0;    // dead slots below L waiting: ring positions [hh, ht)
  int th = 0, tt = 0;    // live slots at or above L waiting: [th, tt)
  for (;;) {
    while (ht - hh < kHoleBatch && hp < L) {
      ht = scan(hp, L, true, sH, kRingH - 1, &s_cnt[0]);
      hp += kScanTile;
    }
    while (tt - th < ht - hh && tp < tail) {
      tt = scan(tp, tail, false, sT, kRingT - 1, &s_cnt[1]);
      tp += kScanTile;
    }
    const int m = min(ht - hh, tt - th);
    if (m == 0) break;
    // the moves of the per-carrier fields read and write with the non-temporal hint: each
    // is touched once, and its scattered writes then leave the cache to the step kernel's
    // data (plain accesses took 21.6 instead of 19.0 ms per batched run); a score row's
    // elements share cache lines, so they move with plain accesses (with the hint the
    // causal replay's compactions took three times as long)
    auto mv = [&](auto* p, int64_t d, int64_t s) {
      __builtin_nontemporal_store(__builtin_nontemporal_load(&p[s]), &p[d]);
    };
    for (int i = tid; i < m; i += kCompactBlock) {
      const int64_t src = base + sT[(th + i) & (kRingT - 1)];
      const int64_t dst = base + sH[(hh + i) & (kRingH - 1)];
      mv(gz, dst, src);
      mv(gmu, dst, src);
      mv(a.E, dst, src);
      mv(a.uid, dst, src);
      mv(a.flags, dst, src);
      if (a.ev) mv(a.ev, dst, src);
      if (a.w) mv(a.w, dst, src);
      if (a.S)
        for (int k = 0; k < a.K; ++k) a.S[dst * a.K + k] = a.S[src * a.K + k];
      if (a.r) mv(a.r, dst, src);
    }
    hh += m;
    th += m;
    __syncthreads();  // the moved ring entries are read before later rounds reuse them
  }
  if (tid == 0) {
    a.slab_tail[slab] = L;
    a.slab_dead[slab] = 0;
  }
}

__global__ void k_fill32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_convert(const uint64_t* dens, int64_t nd, const int64_t* cur, int64_t nc,
                          double* dout, double* cout, double dscale) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd || i < nc;
       i += stride) {
    if (dout && i < nd) dout[i] = (double)dens[i] * dscale;
    if (cout && i < nc) cout[i] = (double)cur[i] * 0x1p-32;
  }
}

template <typename F, int T, int MODE>
static void launch_mode(const StepArgs& a, const StepLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((k_step<F, T, MODE>), dim3(L.grid), dim3(L.block), L.lds, s, a);
}

// the launch modes that are instantiated: debug x density placement x tables x weights
using StepModes = std::integer_sequence<int, 0, 1, 4, 5, 8, 9, 12, 13, 16, 17, 20, 21, 24, 25,
                                        28, 29, 32, 33, 64, 128>;

template <typename F, int T, int... Ms>
static hipError_t launch_any(const StepArgs& a, int mode, const StepLaunch& L, hipStream_t s,
                             std::integer_sequence<int, Ms...>) {
  const bool found = ((mode == Ms ? (launch_mode<F, T, Ms>(a, L, s), true) : false) || ...);
  return found ? hipGetLastError() : hipErrorInvalidValue;
}

template <typename F, int T>
static hipError_t launch_prec(const StepArgs& a, int mode, const StepLaunch& L, hipStream_t s) {
  return launch_any<F, T>(a, mode, L, s, StepModes{});
}

size_t step_static_lds() {
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_step<double, kMaxSub, kModeDebug>)) != hipSuccess)
    return 8192;
  return fa.sharedSizeBytes;
}

template <typename F, int T, int... Ms>
static hipError_t raise_lds_all(size_t bytes, std::integer_sequence<int, Ms...>) {
  hipError_t e = hipSuccess;
  for (const void* f : {reinterpret_cast<const void*>(&k_step<F, T, Ms>)...})
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return e;
}

template <typename F, int T>
static hipError_t raise_lds(size_t bytes) {
  return raise_lds_all<F, T>(bytes, StepModes{});
}

hipError_t set_step_lds_limit(size_t bytes) {
  hipError_t e = raise_lds<float, 1>(bytes);
  if (e == hipSuccess) e = raise_lds<float, 2>(bytes);
  if (e == hipSuccess) e = raise_lds<double, 1>(bytes);
  if (e == hipSuccess) e = raise_lds<double, 2>(bytes);
  return e;
}

hipError_t launch_step(const StepArgs& a, bool fp64, const StepLaunch& L, hipStream_t s) {
  const bool dens_any = a.sub_dens_on[0] || (a.n_sub > 1 && a.sub_dens_on[1]);
  int mode = (a.debug ? kModeDebug : 0) | (dens_any && !a.dens_lds ? kModeDensGlobal : 0) |
             (a.etab_words > 0 ? kModeTab : 0) | (a.wt ? kModeWt : 0) |
             (dens_any && a.dens16 ? kModeDens16 : 0);
  // the whole-tree adjoint's passes (plain runs only: the host checks)
  if (a.adj_pass) mode = a.adj_pass == 1 ? kModeRet : kModeScore;
  if (L.ev[0]) (void)hipEventRecord(L.ev[0], s);
  hipError_t e;
  if (a.n_sub == 2)
    e = fp64 ? launch_prec<double, 2>(a, mode, L, s) : launch_prec<float, 2>(a, mode, L, s);
  else
    e = fp64 ? launch_prec<double, 1>(a, mode, L, s) : launch_prec<float, 1>(a, mode, L, s);
  if (L.ev[1]) (void)hipEventRecord(L.ev[1], s);
  return e;
}

hipError_t launch_compact(const CompactArgs& a, bool fp64, hipStream_t s) {
  if (a.n_slabs <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(k_compact<double>, dim3(a.n_slabs), dim3(kCompactBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_compact<float>, dim3(a.n_slabs), dim3(kCompactBlock), 0, s, a);
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
                          double* dout, double* cout, double dscale, hipStream_t s) {
  const int64_t n = nd > nc ? nd : nc;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, s, dens, nd, cur, nc,
                     dout, cout, dscale);
  return hipGetLastError();
}

}  // namespace pic
