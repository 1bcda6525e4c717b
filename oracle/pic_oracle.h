/* CPU oracle for the spin-dependent hot-electron particle-in-cell step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow FP64 reference written from
 * Nenno, Rethfeld and Schneider, arXiv:1807.04733, Sec. III.A (Eqs. 10-19).  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or table generator with the device library.
 *
 * Units: z in nm, t in fs, velocities in nm/fs, energies as uint32 with LSB 2^-30 eV.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_C_INJECTED = 0, ORC_C_EV_EE, ORC_C_EV_EL, ORC_C_SPAWNED, ORC_C_ABSORBED,
  ORC_C_SEC_ABSORBED, ORC_C_TRANSMIT, ORC_C_REFL_IF, ORC_C_REFL_SURF, ORC_C_ALIVE, ORC_C_E_ABSORBED,
  ORC_C_W_INJECTED,           /* sum of the primaries' weights, 2^-16 units (Eq. 10) */
  ORC_NCOUNTERS
};

typedef struct {
  int32_t n_layers, n_channels, n_ttables, t_entries;
  const double*  z_bound;     /* [L+1] */
  const int32_t* ch_of;       /* [L][2] channel of (layer, global spin) */
  const double*  v;           /* [C] nm/fs */
  const double*  inv_tau0;    /* [C] 1/fs */
  const double*  inv_tau_el;  /* [L] 1/fs */
  const double*  P0;          /* [L] */
  const double*  T;           /* [NT][TE] */
  const int32_t* tt_of;       /* [L-1][2][2] */
  double T_scale;
  double src_z_lo, src_z_hi, src_lambda, src_cd, src_up_frac;
  uint32_t src_e_lo[2], src_e_span[2];
  const int64_t* sched;       /* [n_steps] */
  uint64_t root_offset;
  int32_t nz;
  double inv_dz;
  /* optional energy-dependent channels (Fig. 1: v(E), tau(E)): with e_nodes > 0 the speed
   * of channel c is the linear interpolation of v_node[c][.] and 1/tau_in is inv_tau0[c]
   * times the interpolation of r_node[c][.] (tau_exp is then ignored); nodes at
   * E = k / e_scale eV, k < e_nodes, clamped beyond the last */
  int32_t e_nodes;
  double e_scale;
  const double* v_node;       /* [C][e_nodes] nm/fs */
  const double* r_node;       /* [C][e_nodes] relative inelastic rate */
  /* optional superparticle weights (Eq. 10): with w_nodes > 0 a primary of spin s and
   * initial energy E0 carries the weight interpolated from w_node[s][.] (nodes at
   * E = k / w_scale eV, clamped beyond the last), held as the integer rint(w 2^16); its
   * secondaries inherit it.  w_nodes = 0: weight 1 */
  int32_t w_nodes;
  double w_scale;
  const double* w_node;       /* [2][w_nodes] */
} orc_instance;

typedef struct {
  int32_t n_instances;
  const orc_instance* inst;
  uint64_t seed;
  double dt;
  int32_t n_steps;
  int32_t tau_exp;            /* 0: tau = tau0, 2: tau = tau0 (1 eV/E)^2 */
  uint32_t e_min_fx;
  int32_t secondaries;
  int32_t state_fp64;         /* 0: positions/directions stored as binary32 */
  int32_t n_ebins;
  const uint32_t* e_edges;    /* [n_ebins] lower edges */
  int32_t dens_stride, cur_stride;
  int64_t root_lo, root_hi;   /* simulate local roots in [lo, hi) of every instance; hi<0: all */
  int32_t n_threads;          /* 0: OpenMP default */
  int32_t absorb_next;        /* 0: a product below E_min is removed at once; 1: carriers
                                 below E_min live on and are removed at their next
                                 scattering event (Sec. III.A, lowest energy bin) */
  int32_t weighted;           /* 1: the moments are sums over carriers of their weight
                                 (density and generation label in 2^-16 units, current
                                 rint(v cos(theta) w 2^32)); 0: plain counts */
  /* Scripted random numbers (white-box tests): n_script entries of 8 words, a Philox
   * counter (4 words) and the 4 words to return for it instead of the generator's; every
   * counter not listed draws from Philox as usual.  NULL / 0: off. */
  const uint32_t* script;
  int64_t n_script;
} orc_problem;

typedef struct {
  /* bins, flattened over instances in order: dens [n_dslots][nz][NE][2], cur [n_cslots][nz][2] */
  uint64_t* dens;
  int64_t*  cur;              /* fixed point, 2^-32 nm/fs per unit */
  int64_t*  counters;         /* [n_steps][ORC_NCOUNTERS] */
  /* optional per-particle records of every particle ever created (NULL to skip) */
  int64_t   rec_cap;
  int64_t   n_rec;            /* out */
  uint64_t* rec_uid;
  double*   rec_z;
  double*   rec_mu;
  uint32_t* rec_E;
  int32_t*  rec_layer;
  int32_t*  rec_spin;
  int32_t*  rec_gen;
  int32_t*  rec_dead;         /* step of absorption, -1 if alive at the end */
  int32_t*  rec_inst;
  int32_t*  rec_ev;           /* [4] per record: events, transmissions, reflections, spawns */
  uint32_t* rec_w;            /* weight in 2^-16 units (may be NULL) */
  /* optional generation moment (NULL to skip): sum of the generation label (1: primary,
   * each secondary its parent's + 1) per (density slot, depth, spin), layout
   * [n_dslots][nz][2] per instance, instances concatenated; taken with the density */
  uint64_t* gen;
  /* optional likelihood-ratio gradient (NULL to skip); see orc_run's gradient section */
  const double* g_dens;       /* same layout as dens */
  const double* g_cur;        /* same layout as cur (per unit of nm/fs) */
  double*   grad;             /* [n_channels + n_ttables*t_entries] of instance 0's layout */
  int32_t   grad_per_tree;    /* 0: causal score; 1: whole-tree return */
} orc_output;

/* Philox4x32 with 10 rounds (Salmon et al., SC'11), written from the published definition. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Run the whole problem; returns 0 on success, nonzero on invalid input or record overflow. */
int orc_run(const orc_problem* p, orc_output* o);

#ifdef __cplusplus
}
#endif
#endif
