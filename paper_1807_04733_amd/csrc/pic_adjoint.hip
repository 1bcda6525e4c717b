// Likelihood-ratio adjoint of the particle-in-cell step (gfx950).
//
// The gradient of L = sum(g_dens * density) + sum(g_cur * current) with respect to
// theta = (ln tau0 per channel, every transmission-table node) is the expectation of
// (deposit weight) x (score of the random decisions that led to the deposit).  The random
// decisions of the method (arXiv:1807.04733, Sec. III.A) whose probabilities depend on
// theta are the scattering Bernoulli draw with p = 1 - exp(-dt/tau_eff) (Eq. 2), the
// elastic / inelastic channel choice (Eqs. 5, 8) and the transmission draw at every
// interface hit; their scores are d/dtheta of the log-probability of the outcome taken.
//
// The replay re-runs the forward dynamics bit for bit (same Philox words, same order of
// binary64 operations) and never stores anything from the forward run.
//
//   ADJ = 1  causal estimator: every carrier owns a score row S[K] in HBM that it
//            inherits from its parent at birth; a deposit adds g * weight * S.
//   ADJ = 2  whole-tree estimator, pass 1: the return R of each primary tree
//            (sum of g * weight over all deposits of the tree).
//   ADJ = 3  whole-tree estimator, pass 2: every score term times its tree's R.
//
// The non-event term of a carrier, +x_in per step (x_in = dt/tau_inelastic), is constant
// while neither its energy nor its layer changes, so it is accumulated lazily: the step
// from which terms are still pending lives in spare bits of the flags word and the
// pending m * x_in is folded in only when the carrier's state changes or it deposits
// with g != 0.  A carrier that does neither touches no adjoint memory in that step.
#include "pic_device.h"

#pragma clang fp contract(off)

namespace pic {

constexpr int kSlowQ = (int)(kSlowQueueBytes / 4);  // general-path slots per wave queue
// bytes per wave of the copies of the queued carriers' stored state
template <typename F>
constexpr size_t kAdjStageBytes = (size_t)kSlowQ * (2 * sizeof(F) + 20);

// Per-lane adjoint bookkeeping of one carrier.
struct AdjLane {
  int64_t row;      // slot of the carrier (its score row / return)
  uint32_t root;    // global root id (index of its tree's return)
  double R;         // its tree's return (ADJ 3), loaded on first use
  bool haveR;
};

template <int ADJ>
struct AdjOps {
  const AdjArgs& A;
  double* s_grad;

  __device__ __forceinline__ double tree_return(AdjLane& L) const {
    if (!L.haveR) {
      L.R = A.R[L.root];
      L.haveR = true;
    }
    return L.R;
  }
  // add score v to parameter k of the carrier
  __device__ __forceinline__ void score(AdjLane& L, int k, double v) const {
    if (ADJ == 1) A.S[L.row * A.K + k] += v;
    if (ADJ == 3) atomicAdd(&s_grad[k], v * tree_return(L));
  }
  // fold the pending non-event terms of steps nf .. upto-1 into the score
  __device__ __forceinline__ void flush(AdjLane& L, uint32_t& fl, uint32_t upto, int chan,
                                        double x_in) const {
    const uint32_t nf = nf_of(fl);
    if (upto > nf) {
      if (ADJ != 2) score(L, chan, (double)(upto - nf) * x_in);
      fl = with_nf(fl, upto);
    }
  }
};

__device__ __forceinline__ double x_inelastic(const StepArgs& a, const DevInst& I, const double* et,
                                              uint32_t fl, uint32_t E) {
  const int l = layer_of(fl), s = (int)(fl & kSpinMask);
  return a.dt * inel_rate_at(I, et, a.tau_exp2 != 0, l, s, E);
}

// Interface decisions of a half step become score terms on the table nodes.
template <int ADJ>
struct HitScore {
  const AdjOps<ADJ>& ops;
  const StepArgs& a;
  const DevInst& I;
  const double* et;
  AdjLane& L;
  uint32_t& fl;
  uint32_t E;
  uint32_t upto;
  __device__ __forceinline__ void operator()(int tab, int layer, double T, bool go) const {
    if (ADJ == 2) return;
    const int s = (int)(fl & kSpinMask);
    const uint32_t flx = (fl & ~(kLayerMask << kLayerShift)) | ((uint32_t)layer << kLayerShift);
    ops.flush(L, fl, upto, I.chi[layer][s], x_inelastic(a, I, et, flx, E));
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
    const int base = ops.A.n_ch + tab * TE + k0;
    if (go) {
      ops.score(L, base, w0 / T);
      if (w1 != 0.0) ops.score(L, base + 1, w1 / T);
    } else {
      ops.score(L, base, -w0 / (1.0 - T));
      if (w1 != 0.0) ops.score(L, base + 1, -w1 / (1.0 - T));
    }
  }
};

// Deposit weight of a carrier at the end of step n: g of its density bin (weight 1) plus
// g of its current bin times v*cos(theta) (the fixed-point value the forward deposits).
// Weighted superparticles (Eq. 10) deposit their weight w (wfx in 2^-16 units): the
// density term is g w and the current value rint(v cos(theta) w 2^32).
__device__ __forceinline__ double deposit_weight(const AdjArgs& A, const DevInst& I,
                                                 const double* et, double z, double mu, uint32_t E,
                                                 uint32_t fl, uint32_t wfx, const uint32_t* s_edges,
                                                 const double* s_gcur) {
  const StepArgs& a = A.s;
  int zb = (int)floor(z * I.inv_dz);
  zb = zb < 0 ? 0 : (zb > I.nz - 1 ? I.nz - 1 : zb);
  const int s = (int)(fl & kSpinMask);
  double g = 0.0;
  if (a.dens_on && A.g_dens) {
    const int eb = a.n_ebins > 1 ? energy_bin(s_edges, a.n_ebins, E) : 0;
    const double gd =
        A.g_dens[I.dens_off + (((int64_t)a.dens_slot * I.nz + zb) * a.n_ebins + eb) * 2 + s];
    g += a.wt ? gd * ((double)wfx * 0x1p-16) : gd;
  }
  if (a.cur_on && A.g_cur) {
    const double gc = s_gcur[zb * 2 + s];
    if (gc != 0.0) {
      const double v = speed_at(I, et, layer_of(fl), s, E);
      const long long val = a.wt ? cur_fixed_w(v, mu, wfx) : cur_fixed(v, mu);
      g += gc * ((double)val * 0x1p-32);
    }
  }
  return g;
}

template <int ADJ>
__device__ __forceinline__ void on_deposit(const AdjOps<ADJ>& ops, const StepArgs& a,
                                           const DevInst& I, const double* et, AdjLane& L,
                                           uint32_t& fl, uint32_t E, double g, uint32_t step) {
  if (g == 0.0) return;
  const AdjArgs& A = ops.A;
  if (ADJ == 1) {
    ops.flush(L, fl, step + 1, I.chi[layer_of(fl)][fl & kSpinMask], x_inelastic(a, I, et, fl, E));
    for (int k = 0; k < A.K; ++k) atomicAdd(&ops.s_grad[k], g * A.S[L.row * A.K + k]);
  }
  if (ADJ == 2) A.r[L.row] += g;
}

// Append a carrier behind the slab's tail: one LDS atomic per wave, positions by ballot.
__device__ __forceinline__ int append_slot(bool want, int* s_app, int tail0) {
  const uint64_t m = __ballot(want);
  int off = 0;
  if (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    if (__lane_id() == leader) off = atomicAdd(s_app, __popcll(m));
    off = __shfl(off, leader);
  }
  return tail0 + off + __popcll(m & lanes_below());
}

template <typename F, int ADJ>
__global__ void __launch_bounds__(256, 4) k_adj(AdjArgs A) {
  const StepArgs& a = A.s;
  // dynamic LDS: this step's slice of dL/d(current) for the workgroup's instance, one
  // general-path slot queue per wave, then the instance's energy tables (if any)
  extern __shared__ double s_gcur[];
  uint32_t* s_slow =
      (uint32_t*)((unsigned char*)s_gcur + (((size_t)a.lds_cur_words * 8 + 15) & ~(size_t)15));
  double* const s_etab = (double*)((unsigned char*)s_slow + (blockDim.x / 64) * kSlowQueueBytes);
  const double* const et = a.etab ? s_etab : nullptr;
  // then, per wave, copies of the stored state of the carriers in its queue (z, cos(theta),
  // E, flags, weight, uid), so that their general pass reads LDS instead of HBM
  unsigned char* const s_stage =
      (unsigned char*)s_etab + (((a.etab ? (size_t)a.etab_words * 8 : 0) + 15) & ~(size_t)15);
  const bool tau2 = a.tau_exp2 != 0;
  __shared__ DevInst s_inst;
  __shared__ double s_grad[kMaxK];
  __shared__ uint32_t s_edges[PIC_MAX_EBINS];
  __shared__ int s_slab, s_app, s_dead;
  const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
  for (int i = tid; i < A.K; i += blockDim.x) s_grad[i] = 0.0;
  for (int i = tid; i < a.n_ebins; i += blockDim.x) s_edges[i] = a.e_edges[i];
  F* gz = (F*)a.z;
  F* gmu = (F*)a.mu;
  const uint32_t step = (uint32_t)a.step;
  // stamp of every z this step stores (0 when the step ends a write-back period)
  const uint32_t z_next = a.z_write ? 0u : (uint32_t)a.z_phase + 1u;
  uint32_t* SQ = s_slow + wave * kSlowQ;
  F* const st_z = (F*)(s_stage + (size_t)wave * kAdjStageBytes<F>);
  F* const st_mu = st_z + kSlowQ;
  uint32_t* const st_E = (uint32_t*)(st_mu + kSlowQ);
  uint32_t* const st_fl = st_E + kSlowQ;
  uint32_t* const st_w = st_fl + kSlowQ;
  uint64_t* const st_u = (uint64_t*)(st_w + kSlowQ);
  const AdjOps<ADJ> ops{A, s_grad};
  int cur_inst = -1;
  bool bad = false;

  for (;;) {
    if (tid == 0) s_slab = atomicAdd(&a.queue[a.step], 1);
    __syncthreads();
    const int slab = s_slab;
    if (slab >= a.n_slabs) break;
    const int inst = a.slab_inst[slab];
    if (inst != cur_inst) {
      __syncthreads();
      const uint4* src = (const uint4*)&a.inst[inst];
      uint4* dst = (uint4*)&s_inst;
      for (int i = tid; i < a.inst_bytes / 16; i += blockDim.x) dst[i] = src[i];
      if (a.cur_on && A.g_cur) {
        const DevInst& Ig = a.inst[inst];
        const double* gsl = A.g_cur + Ig.cur_off + (int64_t)a.cur_slot * Ig.nz * 2;
        for (int i = tid; i < Ig.nz * 2; i += blockDim.x) s_gcur[i] = gsl[i];
      }
      if (a.etab) {
        const DevInst& G = a.inst[inst];
        const int n = 2 * (int)G.n_ch * G.e_nodes;
        const double* tsrc = a.etab + G.etab_off;
        for (int i = tid; i < n; i += blockDim.x) s_etab[i] = tsrc[i];
      }
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
    int sn = 0;  // wave-uniform fill of this wave's general-path queue

    // ---------------------------------------------------------------- general path
    // The whole replayed step of one carrier with its score terms.  All lanes of the wave
    // call it together; lanes with nothing to do pass a dead carrier.
    auto general = [&](bool is_new, int64_t gi, double z, double mu, uint32_t E, uint32_t fl,
                       uint32_t lo, uint32_t hi, uint32_t wfx) __attribute__((always_inline)) {
      const bool alive0 = !(fl & kDead);
      bool died = false;
      AdjLane L{gi, lo, 0.0, false};
      // pass 2: the tree's return, loaded before the half step so that its latency
      // overlaps the transport arithmetic (score terms need it)
      if (ADJ == 3 && alive0) {
        L.R = A.R[lo];
        L.haveR = true;
      }
      const double mu_in = mu;
      const uint32_t E_in = E, fl_in = fl;
      if (alive0) {
        HitCounts hc{0, 0, 0};
        {
          const HitScore<ADJ> hs{ops, a, I, et, L, fl, E, step};
          half_push(I, z, mu, fl, E, lo, hi, step, kTagHalf1, a.h, a.key0, a.key1, hc, bad, et,
                    hs);
        }
        const int l = layer_of(fl);
        const int s = (int)(fl & kSpinMask);
        const double itel = I.lay[l].z;
        const double inel = inel_rate_at(I, et, tau2, l, s, E);
        const double rate = inel + itel;
        const double x = a.dt * rate;
        const double x_in = a.dt * inel;
        const double u0 = u01(decide_word(lo, hi, step, a.key0, a.key1));
        bool event;
        if (u0 >= x) event = false;
        else if (x >= 0x1p-20 && u0 < x - 0.5 * x * x) event = true;
        else event = u0 < -expm1(-x);
        if (event) {
          // the event's own words: channel (y), new direction (z), energy split (w)
          const uint4 w = philox10(lo, hi, step, kTagScat, a.key0, a.key1);
          const int c = I.chi[l][s];
          ops.flush(L, fl, step, c, x_in);
          const double prob = -expm1(-x);
          if (ADJ != 2) ops.score(L, c, -x_in * exp(-x) / prob);
          // removal at the next event (lowest energy bin): no channel choice follows
          const bool removed = a.absorb_next && E < a.e_min;
          if (removed) died = true;
          const bool elastic = !removed && itel > 0.0 && u01(w.y) < itel / rate;
          if (ADJ != 2 && itel > 0.0 && !removed)
            ops.score(L, c, elastic ? x_in / x : -1.0 + x_in / x);
          fl = with_nf(fl, step + 1);
          if (!removed) mu = to_store<F>(dircos(w.z));
          if (!elastic && !removed) {
            const uint32_t E1 = __umulhi(w.w, E);
            const uint32_t E2 = E - E1;
            E = E1;
            if (a.secondaries && (E2 >= a.e_min || a.absorb_next)) {
              // the newborn: slot now, score row / return inherited, second half step
              const int cpos = append_slot(true, &s_app, tail0);
              if (cpos < cap) {
                const int64_t cg = base + cpos;
                const uint4 sw = philox10(lo, hi, step, kTagSpawn, a.key0, a.key1);
                double cz = z;
                double cmu = to_store<F>(dircos(sw.x));
                const uint32_t cs = u01(sw.y) < I.lay[l].w ? 0u : 1u;
                uint32_t lin = sw.z;
                if (lin == 0u || lin == hi) {
                  lin = sw.w | 1u;
                  if (lin == hi) lin ^= 2u;
                }
                uint32_t gen = (fl >> kGenShift) & kGenMask;
                gen = gen < 255u ? gen + 1u : 255u;
                uint32_t cfl = with_nf(cs | ((uint32_t)l << kLayerShift) | (gen << kGenShift) |
                                           (z_next << kStampShift),
                                       step + 1);
                if (ADJ == 1)
                  for (int k = 0; k < A.K; ++k) A.S[cg * A.K + k] = A.S[gi * A.K + k];
                if (ADJ == 2) A.r[cg] = 0.0;
                AdjLane CL{cg, lo, L.R, L.haveR};
                HitCounts chc{0, 0, 0};
                {
                  const HitScore<ADJ> hs{ops, a, I, et, CL, cfl, E2, step + 1};
                  half_push(I, cz, cmu, cfl, E2, lo, lin, step, kTagHalf2, a.h, a.key0, a.key1,
                            chc, bad, et, hs);
                }
                cz = to_store<F>(cz);
                const double g = deposit_weight(A, I, et, cz, cmu, E2, cfl, wfx, s_edges, s_gcur);
                on_deposit<ADJ>(ops, a, I, et, CL, cfl, E2, g, step);
                gz[cg] = (F)cz;
                gmu[cg] = (F)cmu;
                a.E[cg] = E2;
                a.uid[cg] = (uint64_t)lo | ((uint64_t)lin << 32);
                a.flags[cg] = cfl;
                if (a.wt) a.wt[cg] = wfx;  // a secondary carries its parent's weight
              } else {
                atomicOr(a.status, kStOverflow);
              }
            }
            if (E1 < a.e_min && !a.absorb_next) died = true;
          }
        }
        if (!died) {
          {
            const HitScore<ADJ> hs{ops, a, I, et, L, fl, E, step + 1};
            half_push(I, z, mu, fl, E, lo, hi, step, kTagHalf2, a.h, a.key0, a.key1, hc, bad, et,
                      hs);
          }
          z = to_store<F>(z);
          const double g = deposit_weight(A, I, et, z, mu, E, fl, wfx, s_edges, s_gcur);
          on_deposit<ADJ>(ops, a, I, et, L, fl, E, g, step);
        } else {
          z = to_store<F>(z);
          fl |= kDead;
          if (ADJ == 2) {
            const double r = A.r[gi];
            if (r != 0.0) atomicAdd(&A.R[lo], r);
          }
        }
        // z is stored below: the stamp says at which step of the write-back period
        fl = (fl & ~(kStampMask << kStampShift)) | (died ? 0u : z_next << kStampShift);
        if (is_new) {
          gz[gi] = (F)z;
          gmu[gi] = (F)mu;
          a.E[gi] = E;
          a.flags[gi] = fl;
          a.uid[gi] = (uint64_t)lo | ((uint64_t)hi << 32);
        } else {
          gz[gi] = (F)z;
          if (mu != mu_in) gmu[gi] = (F)mu;
          if (E != E_in) a.E[gi] = E;
          if (fl != fl_in) a.flags[gi] = fl;
        }
      }
      const uint64_t md = __ballot(died);
      if (md && lane == __ffsll((unsigned long long)md) - 1) atomicAdd(&s_dead, __popcll(md));
    };

    auto wave_sync = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // finish the top n queued general-path slots (their stored state from the LDS copy)
    auto drain_slow = [&](int n) {
      wave_sync();
      const bool act = lane < n;
      const int q = sn - n + lane;
      const uint32_t t = act ? SQ[q] : 0u;
      sn -= n;
      const int64_t g = base + t;
      uint32_t fl = kDead, E = 0, lo = 0, hi = 0, wfx = 1u << 16;
      double z = 0.0, mu = 0.0;
      if (act) {
        fl = st_fl[q];
        wfx = st_w[q];
        z = (double)st_z[q];
        mu = (double)st_mu[q];
        E = st_E[q];
        const uint64_t u = st_u[q];
        lo = (uint32_t)u;
        hi = (uint32_t)(u >> 32);
        const int d = a.z_phase - (int)((fl >> kStampShift) & kStampMask);
        if (d > 0) {
          const double v = speed_at(I, et, layer_of(fl), (int)(fl & kSpinMask), E);
          z = replay_flights<F>(z, (v * mu) * a.h, d);
        }
      }
      general(false, g, z, mu, E, fl, lo, hi, wfx);
      wave_sync();
    };

    // next slot of this lane, fetched one iteration ahead (as in the forward step), with
    // its partial return in pass 1 of the whole-tree estimator: only the carrier in the
    // slot changes it, so the prefetched value is current when the lane gets there
    F nz = 0, nmu = 0;
    uint32_t nE = 0, nfl = kDead, nw = 1u << 16;
    uint64_t nu = 0;
    double nr = 0.0;
    auto fetch = [&](int t) {
      if (t < tail0) {
        const int64_t g = base + t;
        nfl = a.flags[g];
        nz = gz[g];
        nmu = gmu[g];
        nE = a.E[g];
        nu = a.uid[g];
        if (a.wt) nw = a.wt[g];
        if (ADJ == 2) nr = A.r[g];
      } else {
        nfl = kDead;
      }
    };
    fetch(wave * 64 + lane);
    for (int tb = wave * 64; tb < total; tb += blockDim.x) {
      const int t = tb + lane;
      const F rz = nz, rmu = nmu;
      const uint32_t rE = nE, rfl = nfl, rw = nw;
      const uint64_t ru = nu;
      const double rr = nr;
      fetch(t + (int)blockDim.x);
      const bool have = t < total;
      const bool from_soa = have && t < tail0;
      const bool is_new = have && !from_soa;

      // ---- common step: no boundary in either half step, a draw at or above x >= p
      // (certainly no event) and, for the causal estimator, a deposit weight of 0: no
      // score term at all; identical arithmetic to the general path
      bool slow = false;
      if (from_soa && !(rfl & kDead)) {
        const int l = layer_of(rfl), s = (int)(rfl & kSpinMask);
        const LayCache c = load_lay<true>(I, et, tau2, l, s, rE);
        const double mu = (double)rmu;
        const uint32_t st = (rfl >> kStampShift) & kStampMask;
        const double z0 = replay_flights<F>((double)rz, (c.v * mu) * a.h, a.z_phase - (int)st);
        const double zm = z0 + (c.v * mu) * a.h;
        const uint32_t wd = decide_word((uint32_t)ru, (uint32_t)(ru >> 32), step, a.key0, a.key1);
        const double x = a.dt * (c.itau + I.lay[l].z);
        const double ze = zm + (c.v * mu) * a.h;
        slow = zm > c.zhi || zm < c.zlo || u01(wd) < x || ze > c.zhi || ze < c.zlo;
        if (!slow) {
          const double zs = to_store<F>(ze);
          const int64_t gi = base + t;
          if (ADJ != 3) {
            const double g = deposit_weight(A, I, et, zs, mu, rE, rfl, rw, s_edges, s_gcur);
            if (ADJ == 1 && g != 0.0) slow = true;
            if (ADJ == 2 && g != 0.0) A.r[gi] = rr + g;
          }
          if (!slow && a.z_write) {
            gz[gi] = (F)zs;
            if (st) a.flags[gi] = rfl & ~(kStampMask << kStampShift);
          }
        }
      }
      // ---- new primaries take their slot first, so that their score row exists
      if (__ballot(is_new)) {
        const int newpos = append_slot(is_new, &s_app, tail0);
        int64_t gi = base + t;
        double z = 0.0, mu = 0.0;
        uint32_t E = 0, fl = kDead, lo = 0, wfx = 1u << 16;
        if (is_new) {
          gi = base + newpos;
          if (newpos >= cap) {
            atomicOr(a.status, kStOverflow);
          } else {
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
            fl = with_nf(s | ((uint32_t)l << kLayerShift) | (1u << kGenShift), step);
            lo = root;
            if (a.wt) {
              wfx = primary_weight(I, a.etab + I.etab_off + 2 * (int)I.n_ch * I.e_nodes, (int)s, E);
              a.wt[gi] = wfx;
            }
            if (ADJ == 1)
              for (int k = 0; k < A.K; ++k) A.S[gi * A.K + k] = 0.0;
            if (ADJ == 2) A.r[gi] = 0.0;
          }
        }
        general(is_new && newpos < cap, gi, z, mu, E, fl, lo, 0u, wfx);
      }
      // ---- queue the general-path slots
      const uint64_t ms = __ballot(slow);
      if (ms) {
        if (slow) {
          const int q = sn + prefix_count(ms);
          SQ[q] = (uint32_t)t;
          st_z[q] = rz;
          st_mu[q] = rmu;
          st_E[q] = rE;
          st_fl[q] = rfl;
          st_w[q] = rw;
          st_u[q] = ru;
        }
        sn += __popcll(ms);
      }
      if (sn >= 64) drain_slow(64);
    }
    while (sn > 0) drain_slow(sn < 64 ? sn : 64);
    __syncthreads();
    if (tid == 0) {
      int nt = tail0 + s_app;
      if (nt > cap) nt = cap;
      a.slab_tail[slab] = nt;
      a.slab_dead[slab] += s_dead;
    }
  }
  if (bad) atomicOr(a.status, kStHits);
  __syncthreads();
  if (ADJ != 2)
    for (int k = tid; k < A.K; k += blockDim.x)
      if (s_grad[k] != 0.0) atomicAdd(&A.grad[k], s_grad[k]);
}

// After the last step: trees still alive hand in their returns (pass 1), and pending
// non-event terms are folded in (pass 2).
template <typename F, int ADJ>
__global__ void __launch_bounds__(256) k_adj_final(AdjArgs A, uint32_t n_steps) {
  const StepArgs& a = A.s;
  __shared__ double s_grad[kMaxK];
  __shared__ DevInst s_inst;
  const int slab = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < A.K; i += blockDim.x) s_grad[i] = 0.0;
  const int inst = a.slab_inst[slab];
  const uint4* src = (const uint4*)&a.inst[inst];
  uint4* dst = (uint4*)&s_inst;
  for (int i = tid; i < a.inst_bytes / 16; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  const DevInst& I = s_inst;
  const int64_t base = a.slab_base[slab];
  const int tail = a.slab_tail[slab];
  const AdjOps<ADJ> ops{A, s_grad};
  for (int t = tid; t < tail; t += blockDim.x) {
    const int64_t gi = base + t;
    uint32_t fl = a.flags[gi];
    if (fl & kDead) continue;
    const uint32_t lo = (uint32_t)a.uid[gi];
    if (ADJ == 2) {
      const double r = A.r[gi];
      if (r != 0.0) atomicAdd(&A.R[lo], r);
    }
    if (ADJ == 3) {
      AdjLane L{gi, lo, 0.0, false};
      const uint32_t E = a.E[gi];
      // energy tables read from global memory in this one-off pass
      const double* et = a.etab ? a.etab + I.etab_off : nullptr;
      ops.flush(L, fl, n_steps, I.chi[layer_of(fl)][fl & kSpinMask], x_inelastic(a, I, et, fl, E));
    }
  }
  __syncthreads();
  if (ADJ == 3)
    for (int k = tid; k < A.K; k += blockDim.x)
      if (s_grad[k] != 0.0) atomicAdd(&A.grad[k], s_grad[k]);
}

template <typename F>
static hipError_t launch_adj_prec(const AdjArgs& A, int adj, int grid, int block, hipStream_t s) {
  const size_t lds = (((size_t)A.s.lds_cur_words * 8 + 15) & ~(size_t)15) +
                     (size_t)(block / 64) * kSlowQueueBytes +
                     (((A.s.etab ? (size_t)A.s.etab_words * 8 : 0) + 15) & ~(size_t)15) +
                     (size_t)(block / 64) * kAdjStageBytes<F>;
  switch (adj) {
    case 1: hipLaunchKernelGGL((k_adj<F, 1>), dim3(grid), dim3(block), lds, s, A); break;
    case 2: hipLaunchKernelGGL((k_adj<F, 2>), dim3(grid), dim3(block), lds, s, A); break;
    case 3: hipLaunchKernelGGL((k_adj<F, 3>), dim3(grid), dim3(block), lds, s, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjArgs& A, bool fp64, int adj, int grid, int block,
                          hipStream_t s) {
  return fp64 ? launch_adj_prec<double>(A, adj, grid, block, s)
              : launch_adj_prec<float>(A, adj, grid, block, s);
}

hipError_t launch_adjoint_final(const AdjArgs& A, bool fp64, int adj, uint32_t n_steps,
                                hipStream_t s) {
  const int grid = A.s.n_slabs;
  if (grid <= 0) return hipSuccess;
  if (adj == 2) {
    if (fp64) hipLaunchKernelGGL((k_adj_final<double, 2>), dim3(grid), dim3(256), 0, s, A, n_steps);
    else hipLaunchKernelGGL((k_adj_final<float, 2>), dim3(grid), dim3(256), 0, s, A, n_steps);
  } else if (adj == 3) {
    if (fp64) hipLaunchKernelGGL((k_adj_final<double, 3>), dim3(grid), dim3(256), 0, s, A, n_steps);
    else hipLaunchKernelGGL((k_adj_final<float, 3>), dim3(grid), dim3(256), 0, s, A, n_steps);
  } else {
    return hipSuccess;
  }
  return hipGetLastError();
}

}  // namespace pic
