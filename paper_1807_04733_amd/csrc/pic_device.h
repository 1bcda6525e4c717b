// Device helpers shared by the forward step and the adjoint replay: Philox4x32-10, the
// uniform / direction-cosine maps, transmission lookup and the transport half step.
#pragma once
#include "pic_internal.h"

#pragma clang fp contract(off)

namespace pic {

// ------------------------------------------------------------------------- Philox4x32-10
// Salmon et al. (SC'11).  Two 32x32->64 products per round (v_mad_u64_u32); the key is
// wave-uniform, so its Weyl schedule stays in scalar registers.
// Three-input XOR with the round key in a scalar register: gfx950's three-operand
// bitwise op with truth table 0x96 (odd parity), one VALU op instead of two.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}
// Scalar add for the Weyl key schedule; volatile so that the 20 round keys are
// recomputed per call on the scalar unit instead of being kept live in SGPRs.
__device__ __forceinline__ uint32_t key_step(uint32_t k, uint32_t w) {
  uint32_t r;
  asm volatile("s_add_u32 %0, %1, %2" : "=s"(r) : "s"(k), "s"(w) : "scc");
  return r;
}

__device__ __forceinline__ uint4 philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                          uint32_t k0, uint32_t k1) {
  // the key is the same for every lane: keep it (and its schedule) in scalar registers
  k0 = __builtin_amdgcn_readfirstlane(k0);
  k1 = __builtin_amdgcn_readfirstlane(k1);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)x0 * 0xD2511F53ull;
    const uint64_t m1 = (uint64_t)x2 * 0xCD9E8D57ull;
    const uint32_t y0 = xor3_key((uint32_t)(m1 >> 32), x1, k0);
    const uint32_t y2 = xor3_key((uint32_t)(m0 >> 32), x3, k1);
    x1 = (uint32_t)m1;
    x3 = (uint32_t)m0;
    x0 = y0;
    x2 = y2;
    if (r < 9) {
      k0 = key_step(k0, 0x9E3779B9u);
      k1 = key_step(k1, 0xBB67AE85u);
    }
  }
  return make_uint4(x0, x1, x2, x3);
}

// The event-decision words of the step pair (2m, 2m + 1) holding `step`: one generator
// call serves both steps of the pair (word 0 decides step 2m, word 1 step 2m + 1).
__device__ __forceinline__ uint4 decide_pair(uint32_t lo, uint32_t hi, uint32_t step, uint32_t k0,
                                             uint32_t k1) {
  return philox10(lo, hi, step & ~1u, kTagDecide, k0, k1);
}
__device__ __forceinline__ uint32_t decide_word(uint32_t lo, uint32_t hi, uint32_t step,
                                                uint32_t k0, uint32_t k1) {
  const uint4 w = decide_pair(lo, hi, step, k0, k1);
  return (step & 1u) ? w.y : w.x;
}

// uniform on (0,1) and direction cosine on (-1,1): exact in binary64
__device__ __forceinline__ double u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
__device__ __forceinline__ double dircos(uint32_t w) { return ((double)w + 0.5) * 0x1p-31 - 1.0; }

template <typename F>
__device__ __forceinline__ double to_store(double x) { return (double)(F)x; }

__device__ __forceinline__ int layer_of(uint32_t fl) { return (int)((fl >> kLayerShift) & kLayerMask); }

__device__ __forceinline__ double trans_prob(const DevInst& I, int t, uint32_t E) {
  const int TE = I.t_entries;
  const double* tab = I.T + t * TE;
  if (TE == 1) return tab[0];
  const double x = ((double)E * 0x1p-30) * I.T_scale;
  const int k = (int)floor(x);
  if (k >= TE - 1) return tab[TE - 1];
  const double f = x - (double)k;
  return tab[k] + (tab[k + 1] - tab[k]) * f;
}

// Linear interpolation on n equidistant energy nodes at E = k / scale eV, clamped beyond
// the last node (the rule of the transmission tables).
__device__ __forceinline__ double node_interp(const double* tab, int n, double scale, uint32_t E) {
  const double x = ((double)E * 0x1p-30) * scale;
  const int k = (int)floor(x);
  if (k >= n - 1) return tab[n - 1];
  const double f = x - (double)k;
  return tab[k] + (tab[k + 1] - tab[k]) * f;
}

// Speed of the channel of (layer l, spin s) at energy E (Fig. 1(a)); `et` points at the
// instance's energy tables (used only when it has them).
__device__ __forceinline__ double speed_at(const DevInst& I, const double* et, int l, int s,
                                           uint32_t E) {
  if (I.e_nodes) return node_interp(et + I.chi[l][s] * I.e_nodes, I.e_nodes, I.e_scale, E);
  return I.chan[l][s].x;
}

// Inelastic rate 1/tau(E) of (layer l, spin s), Eq. (2) and Fig. 1(b): 1/tau0 times the
// channel's rate table at E, or times (E / 1 eV)^2 (tau2) or 1.
__device__ __forceinline__ double inel_rate_at(const DevInst& I, const double* et, bool tau2,
                                               int l, int s, uint32_t E) {
  if (I.e_nodes) {
    const double r =
        node_interp(et + ((int)I.n_ch + I.chi[l][s]) * I.e_nodes, I.e_nodes, I.e_scale, E);
    return r * I.chan[l][s].y;
  }
  const double E_ev = (double)E * 0x1p-30;
  const double Ek = tau2 ? E_ev * E_ev : 1.0;
  return Ek * I.chan[l][s].y;
}

// Weight of a primary of spin s and initial energy E0 (Eq. 10) in 2^-16 units: the
// interpolation of the spin's row of the instance's weight table (`wrows`, [2][w_nodes]),
// rounded to nearest even; 2^16 without a table.
__device__ __forceinline__ uint32_t primary_weight(const DevInst& I, const double* wrows, int s,
                                                   uint32_t E0) {
  if (!I.w_nodes) return 1u << 16;
  const double w = node_interp(wrows + s * I.w_nodes, I.w_nodes, I.w_scale, E0);
  return (uint32_t)(long long)rint(w * 65536.0);
}

// v cos(theta) of the current moment in 2^-32 nm/fs fixed point, rounded half to even:
// adding 1.5*2^52 (|x| < 2^51) leaves the integer in the low mantissa bits, identical to
// rint().  A weighted carrier (wfx in 2^-16 units, `weighted`) adds rint(v mu w 2^32),
// computed as (v mu wfx) 2^16.
__device__ __forceinline__ long long cur_fixed(double v, double mu) {
  const double vm = v * mu;
  const double sh = vm * 4294967296.0 + 0x1.8p52;
  return __double_as_longlong(sh) - __double_as_longlong(0x1.8p52);
}
__device__ __forceinline__ long long cur_fixed_w(double v, double mu, uint32_t wfx) {
  const double vm = v * mu;
  const double sh = (vm * (double)wfx) * 65536.0 + 0x1.8p52;
  return __double_as_longlong(sh) - __double_as_longlong(0x1.8p52);
}

struct HitCounts {
  uint32_t tr, ri, rs;
};

// Observer of interface decisions (table, layer before the hit, T, transmitted); the
// forward step ignores them, the adjoint turns them into score terms.
struct NoHitObserver {
  __device__ __forceinline__ void operator()(int, int, double, bool) const {}
};

// Transport over half a step.  The common case (no boundary reached) costs one LDS read
// of the layer and one of the channel; boundary handling is a rarely taken loop.
template <class OnHit = NoHitObserver>
__device__ __forceinline__ void half_push(const DevInst& I, double& z, double& mu, uint32_t& fl,
                                          uint32_t E, uint32_t lo, uint32_t hi, uint32_t step,
                                          uint32_t tag, double h, uint32_t k0, uint32_t k1,
                                          HitCounts& hc, bool& bad, const double* et,
                                          OnHit on_hit = OnHit()) {
  int l = layer_of(fl);
  const int s = (int)(fl & kSpinMask);
  const double v = speed_at(I, et, l, s, E);
  double ze = z + (v * mu) * h;
  double zlo = I.lay[l].x, zhi = I.lay[l].y;
  if (ze > zhi || ze < zlo) {
    uint32_t draws = 0;
    for (int hit = 0;; ++hit) {
      const bool up = ze > zhi;
      if (!up && !(ze < zlo)) break;
      if (hit == kMaxHits) {
        bad = true;
        ze = up ? zhi : zlo;
        break;
      }
      const double b = up ? zhi : zlo;
      const bool outer = up ? (l == I.n_layers - 1) : (l == 0);
      if (outer) {
        ze = b - (ze - b);
        mu = -mu;
        ++hc.rs;
        continue;
      }
      const int iface = up ? l : l - 1;
      const int nl = up ? l + 1 : l - 1;
      const int tab = I.tt[iface][up ? 0 : 1][s];
      const double T = trans_prob(I, tab, E);
      bool go;
      if (T >= 1.0) {
        go = true;           // a draw in (0,1) is always below T
      } else if (T <= 0.0) {
        go = false;
      } else {
        const uint4 w = philox10(lo, hi, step, tag + draws, k0, k1);
        go = u01(w.x) < T;
      }
      ++draws;
      on_hit(tab, l, T, go);
      if (go) {
        // speed ratio new/old layer (constant speeds: divided once on the host, the same
        // IEEE quotient)
        const double r = I.e_nodes ? speed_at(I, et, nl, s, E) / speed_at(I, et, l, s, E)
                                   : I.ratio[l][s][up ? 0 : 1];
        ze = b + (ze - b) * r;
        l = nl;
        zlo = I.lay[l].x;
        zhi = I.lay[l].y;
        ++hc.tr;
      } else {
        ze = b - (ze - b);
        mu = -mu;
        ++hc.ri;
      }
    }
    fl = (fl & ~(kLayerMask << kLayerShift)) | ((uint32_t)l << kLayerShift);
  }
  z = ze;
}

// Table values of a carrier's (layer, spin), kept in registers through the step and
// reloaded from LDS only when the carrier changes layer (or energy, with energy tables).
// ET false: v and itau = 1/tau0 of the channel, the energy factor of the rate applied at
// each use (inel_rate).  ET true: v(E) and itau = 1/tau(E) at the carrier's energy.
struct LayCache {
  double zlo, zhi, v, itau;
};

__device__ __forceinline__ LayCache load_lay(const DevInst& I, int l, int s) {
  const double2 C = I.chan[l][s];
  return LayCache{I.lay[l].x, I.lay[l].y, C.x, C.y};
}

template <bool ET>
__device__ __forceinline__ LayCache load_lay(const DevInst& I, const double* et, bool tau2, int l,
                                             int s, uint32_t E) {
  if constexpr (ET)
    return LayCache{I.lay[l].x, I.lay[l].y, speed_at(I, et, l, s, E),
                    inel_rate_at(I, et, tau2, l, s, E)};
  else
    return load_lay(I, l, s);
}

// 1/tau(E) of a cached (layer, spin) at energy E (the same product as inel_rate_at).
template <bool ET>
__device__ __forceinline__ double inel_rate(const LayCache& c, bool tau2, uint32_t E) {
  if constexpr (ET) {
    return c.itau;
  } else {
    const double E_ev = (double)E * 0x1p-30;
    const double Ek = tau2 ? E_ev * E_ev : 1.0;
    return Ek * c.itau;
  }
}

// n straight flights of a whole step each, from a stored position: the common-path step
// (two half-step additions in binary64, then the storage rounding) repeated exactly.
template <typename F>
__device__ __forceinline__ double replay_flights(double z, double vmh, int n) {
  for (int k = 0; k < n; ++k) {
    const double zm = z + vmh;
    z = to_store<F>(zm + vmh);
  }
  return z;
}

// Transport half step with the layer's table values cached (same arithmetic and draws
// as half_push); `on_hit` observes each interface decision as in half_push.
template <bool ET, class OnHit = NoHitObserver>
__device__ __forceinline__ void half_push_c(const DevInst& I, const double* et, bool tau2,
                                            LayCache& c, double& z, double& mu,
                                            uint32_t& fl, uint32_t E, uint32_t lo, uint32_t hi,
                                            uint32_t step, uint32_t tag, double h, uint32_t k0,
                                            uint32_t k1, HitCounts& hc, bool& bad,
                                            OnHit on_hit = OnHit()) {
  double ze = z + (c.v * mu) * h;
  if (ze > c.zhi || ze < c.zlo) {
    int l = layer_of(fl);
    const int s = (int)(fl & kSpinMask);
    uint32_t draws = 0;
    for (int hit = 0;; ++hit) {
      const bool up = ze > c.zhi;
      if (!up && !(ze < c.zlo)) break;
      if (hit == kMaxHits) {
        bad = true;
        ze = up ? c.zhi : c.zlo;
        break;
      }
      const double b = up ? c.zhi : c.zlo;
      const bool outer = up ? (l == I.n_layers - 1) : (l == 0);
      if (outer) {
        ze = b - (ze - b);
        mu = -mu;
        ++hc.rs;
        continue;
      }
      const int iface = up ? l : l - 1;
      const int nl = up ? l + 1 : l - 1;
      const int tab = I.tt[iface][up ? 0 : 1][s];
      const double T = trans_prob(I, tab, E);
      bool go;
      if (T >= 1.0) {
        go = true;
      } else if (T <= 0.0) {
        go = false;
      } else {
        const uint4 w = philox10(lo, hi, step, tag + draws, k0, k1);
        go = u01(w.x) < T;
      }
      ++draws;
      on_hit(tab, l, T, go);
      if (go) {
        if constexpr (ET) {
          const LayCache cn = load_lay<true>(I, et, tau2, nl, s, E);
          ze = b + (ze - b) * (cn.v / c.v);
          c = cn;
        } else {
          ze = b + (ze - b) * I.ratio[l][s][up ? 0 : 1];
          c = load_lay(I, nl, s);
        }
        l = nl;
        ++hc.tr;
      } else {
        ze = b - (ze - b);
        mu = -mu;
        ++hc.ri;
      }
    }
    fl = (fl & ~(kLayerMask << kLayerShift)) | ((uint32_t)l << kLayerShift);
  }
  z = ze;
}

// Number of set bits of a wave mask in the lanes below this one.
__device__ __forceinline__ int prefix_count(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int energy_bin(const uint32_t* edges, int n, uint32_t E) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (edges[mid] <= E) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Energy bin by bucket: the table gives, per bucket of the top bits of E, the bin of the
// bucket's lower end; the few edges inside the bucket are then stepped over.  The same
// result as energy_bin (the last edge <= E, or bin 0 below the first edge).
__device__ __forceinline__ int energy_bin_b(const uint32_t* edges, const uint8_t* bkt, int n,
                                            uint32_t E) {
  int eb = bkt[E >> kEBucketShift];
  while (eb + 1 < n && edges[eb + 1] <= E) ++eb;
  return eb;
}

__device__ __forceinline__ int64_t count_mod(int64_t x, int64_t k, int64_t S) {
  // number of j in [0, x) with j % S == k
  return x > k ? (x - 1 - k) / S + 1 : 0;
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

}  // namespace pic
