/* C ABI of the MI355X hot-electron particle-in-cell library (libpic.so).
 *
 * The library advances the spin-dependent Boltzmann equation for optically excited hot
 * electrons in metallic multilayers with the particle-in-cell method of Nenno, Rethfeld
 * and Schneider (arXiv:1807.04733, Sec. III.A): superparticles (Eq. 10) advanced by the
 * Strang splitting of Eq. (15) -- Source(dt/2) Transport(dt/2) Scattering(dt)
 * Transport(dt/2) Source(dt/2) -- and binned into the moments of Eq. (16) (density per
 * depth, energy and spin) and Eq. (23) (spin current per depth and spin).
 *
 * Conventions
 *   - z in nm, t in fs, speeds in nm/fs; energies above E_F as uint32 fixed point with
 *     an LSB of 2^-30 eV.  Layer boundaries must lie on multiples of 2^-6 nm.
 *   - Global spin s: 0 = up (emitter majority), 1 = down.
 *   - A channel is (material, spin local to the layer); ch_of[l][s] selects the channel
 *     of layer l for global spin s.  Interface k lies between layers k and k+1;
 *     tt_of[k][d][s] is the transmission table for direction d (0: +z, 1: -z).
 *   - Random numbers: Philox4x32-10 keyed by `seed`, counter (uid_lo, uid_hi, step, tag),
 *     one tag per purpose; the event decisions of steps 2m and 2m+1 are words 0 and 1 of
 *     the counter with step field 2m.  Results are a pure function of the inputs,
 *     independent of launch configuration.
 *
 * Memory and streams
 *   - The library never allocates device memory.  The caller supplies one device
 *     workspace of at least pic_workspace_size() bytes (256-byte aligned) and keeps it
 *     alive until pic_destroy(), or sets up with pic_init_static(), which uses a static
 *     array of the library instead.  Output arrays passed to pic_deposit() are caller-owned
 *     device memory.  All device work is enqueued on the HIP stream given to pic_init()
 *     (NULL = the default stream).  pic_init(), pic_inject(), pic_counters(),
 *     pic_backward(), pic_autotune(), pic_time_kernels(), pic_kernel_times() and
 *     pic_destroy() wait for that stream; the other calls only enqueue work.
 *   - A context is not thread-safe; distinct contexts may be used concurrently on
 *     distinct streams.
 *
 * Errors
 *   - Every call returns a pic_status.  PIC_EINVAL: rejected arguments (checked
 *     synchronously, nothing enqueued).  PIC_EHIP: a HIP runtime call failed.
 *     PIC_ECAPACITY / PIC_ESTATE: an asynchronous device condition (particle slots
 *     exhausted -- the excess carriers are dropped and counted, never written out of
 *     bounds; or more than 8 boundary hits in one half step) reported by the next
 *     synchronizing call.  pic_last_error() returns a thread-local message.
 */
#ifndef PIC_H
#define PIC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_LAYERS   16
#define PIC_MAX_CHANNELS 8
#define PIC_MAX_TTABLES  8
#define PIC_MAX_TENTRIES 64
#define PIC_MAX_EBINS    128

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = 1,
  PIC_ENOMEM = 2,     /* workspace too small */
  PIC_ECAPACITY = 3,  /* particle slots exhausted on the device */
  PIC_EHIP = 4,
  PIC_ESTATE = 5      /* call out of order, or a device-side consistency failure */
} pic_status;

/* pic_config.flags */
#define PIC_F_STATE_FP64   1u  /* z and cos(theta) stored as binary64 (else binary32) */
#define PIC_F_SECONDARIES  2u  /* inelastic events lift a secondary carrier (Eq. 6-7) */
#define PIC_F_DEBUG        4u  /* keep per-particle event counts (see pic_layout) */
#define PIC_F_GEN_MOMENT   8u  /* also bin the generation label with the density */
#define PIC_F_ABSORB_NEXT 16u  /* a carrier below E_min is removed at its next scattering
                                  event (Sec. III.A, lowest energy bin) instead of at once;
                                  every secondary is created */
#define PIC_F_WEIGHTS     32u  /* weighted superparticles (Eq. 10): every primary takes a
                                  weight from its instance's weight table at injection,
                                  its secondaries inherit it, and the density, current and
                                  generation moments are weighted sums */

/* per-step counters returned by pic_counters(), [n_steps][PIC_NCOUNTERS] */
enum {
  PIC_C_INJECTED = 0,   /* primaries created at the start of the step (Eq. 17) */
  PIC_C_EV_EE,          /* inelastic (electron-electron) events */
  PIC_C_EV_EL,          /* elastic events */
  PIC_C_SPAWNED,        /* secondaries created */
  PIC_C_ABSORBED,       /* carriers removed after falling below E_min */
  PIC_C_SEC_ABSORBED,   /* secondaries below E_min at birth (never created) */
  PIC_C_TRANSMIT,       /* interface transmissions */
  PIC_C_REFL_IF,        /* interface reflections */
  PIC_C_REFL_SURF,      /* vacuum-surface reflections */
  PIC_C_ALIVE,          /* carriers alive after the step (= sum of the step's density) */
  PIC_C_E_ABSORBED,     /* energy removed with absorbed carriers (fixed point) */
  PIC_C_W_INJECTED,     /* sum of the weights of the primaries created, 2^-16 units
                           (2^16 each without PIC_F_WEIGHTS); the normalisation of
                           Eq. (10) is C = rho_exc / (this sum * 2^-16) */
  PIC_NCOUNTERS
};

/* One layer stack with its parameters (Eqs. 2, 7, 8, 19; Sec. III.A). */
typedef struct {
  int32_t  n_layers;                        /* 1..PIC_MAX_LAYERS */
  int32_t  n_channels;                      /* 1..PIC_MAX_CHANNELS */
  int32_t  n_ttables;                       /* 1..PIC_MAX_TTABLES */
  int32_t  t_entries;                       /* 1 (constant) or 2..PIC_MAX_TENTRIES nodes */
  double   z_bound[PIC_MAX_LAYERS + 1];     /* increasing, multiples of 2^-6 nm */
  int32_t  ch_of[PIC_MAX_LAYERS][2];
  double   v[PIC_MAX_CHANNELS];             /* speed per channel, > 0 */
  double   inv_tau0[PIC_MAX_CHANNELS];      /* 1/tau0; tau = tau0 (1 eV/E)^tau_exp; >= 0 */
  double   inv_tau_el[PIC_MAX_LAYERS];      /* 1/tau_el per layer (0 = no elastic channel) */
  double   P0[PIC_MAX_LAYERS];              /* equilibrium polarisation, Eq. (19), [-1,1] */
  int32_t  tt_of[PIC_MAX_LAYERS - 1][2][2];
  double   T[PIC_MAX_TTABLES][PIC_MAX_TENTRIES]; /* transmission probabilities in [0,1] */
  double   T_scale;                         /* (t_entries-1)/E_table_max, 1/eV */
  /* pump (Eq. 17): depth z0 = lo - lambda*log1p(-u*cd) (lambda > 0) or lo + u*(hi-lo),
   * cd = 1 - exp(-(hi-lo)/lambda); spin up with probability up_frac; energy
   * e_lo[s] + floor(w * e_span[s] / 2^32) for a uniform 32-bit word w. */
  double   src_z_lo, src_z_hi, src_lambda, src_cd, src_up_frac;
  uint32_t src_e_lo[2], src_e_span[2];
  int64_t  n_primaries;                     /* total primaries of this instance */
  uint64_t root_offset;                     /* global id of its first primary */
  int32_t  nz;                              /* depth bins [k/inv_dz, (k+1)/inv_dz) */
  double   inv_dz;
  /* Optional energy-dependent channels (Fig. 1: v(E) and tau(E) per material and spin).
   * e_nodes = 0: speed v[c] and 1/tau_in = inv_tau0[c] (E/1 eV)^tau_exp.  e_nodes in
   * 2..PIC_MAX_TENTRIES: nodes at E = k / e_scale eV (k < e_nodes); the speed of channel c
   * is the linear interpolation of v_node[c][.] (> 0) and 1/tau_in = inv_tau0[c] times the
   * interpolation of r_node[c][.] (>= 0, tau_exp ignored), both clamped to the last node
   * above it (the rule of the transmission tables).  v[] is then unused. */
  int32_t  e_nodes;
  double   e_scale;                         /* 1/eV, > 0 when e_nodes > 0 */
  double   v_node[PIC_MAX_CHANNELS][PIC_MAX_TENTRIES];
  double   r_node[PIC_MAX_CHANNELS][PIC_MAX_TENTRIES];
  /* Superparticle weights (Eq. 10; used with PIC_F_WEIGHTS).  w_nodes = 0: weight 1.
   * w_nodes in 1..PIC_MAX_TENTRIES: a primary of spin s and initial energy E0 weighs the
   * linear interpolation of w_node[s][.] at E0 (nodes at E = k / w_scale eV, clamped to
   * the last; one node: a constant per spin), held as the integer rint(w 2^16).  Values
   * in [2^-16, 2^15]. */
  int32_t  w_nodes;
  double   w_scale;                         /* 1/eV, in [0, 1e8] */
  double   w_node[2][PIC_MAX_TENTRIES];
} pic_instance;

typedef struct {
  int32_t  n_instances;                     /* >= 1 */
  const pic_instance* inst;                 /* host array, copied by pic_init */
  uint64_t seed;
  double   dt;                              /* > 0 */
  int32_t  n_steps;                         /* >= 1 */
  int32_t  tau_exp;                         /* 0 or 2 */
  uint32_t e_min_fx;                        /* carriers below this energy are removed */
  uint32_t flags;                           /* PIC_F_* */
  int32_t  n_ebins;                         /* 1..PIC_MAX_EBINS */
  uint32_t e_edges[PIC_MAX_EBINS];          /* increasing lower edges (last bin open) */
  int32_t  dens_stride, cur_stride;         /* deposit every k-th step (slot n/k) */
  int32_t  slab_primaries;                  /* primaries per slab; 0 = default: with
                                               instances of equal size, a slab count that
                                               is a multiple of the step kernel's resident
                                               workgroups (2 per CU; 4 with an adjoint) at
                                               <= 32768 primaries per slab; else 16384, or
                                               fewer so that there are >= 2048 slabs */
  double   capacity_factor;                 /* slots per primary; 0 = floor(E0max/Emin)+2 */
  int32_t  adjoint;                         /* workspace for pic_backward: 0 none, 1 causal
                                               (K <= 16), 2 whole-tree, 3 both.  Needs equal
                                               table shapes in all instances and
                                               n_steps <= 32767 */
} pic_config;

/* Launch tuning.  Results never depend on it. */
typedef struct {
  int32_t block;          /* threads per workgroup: 64, 128, 256, 512 or 1024 */
  int32_t grid;           /* persistent workgroups per step launch; 0 = 2 x 256 CUs */
  int32_t compact_every;  /* launch the compaction pass every k steps; 0 = never */
  float   compact_frac;   /* compact a slab when dead slots exceed this fraction */
  int32_t use_graph;      /* capture multi-step calls in a hipGraph */
  int32_t z_every;        /* a carrier on the common path (no boundary, no event) stores
                             its z every z_every steps (1..8) and at the end of every
                             pic_step call; in between z is recomputed from the stored
                             value by repeating the straight flights exactly */
  int32_t sub_steps;      /* steps advanced per kernel launch (1 or 2): a carrier that
                             stays on the common path does them from registers, with one
                             pass over its state; z_every is rounded up to a multiple */
} pic_tuning;

/* Where things live inside the workspace (byte offsets), for inspection and tests.
 * The slab table lists each instance's slabs together, instances in decreasing order of
 * primaries per slab times mean initial energy (the order in which slabs are processed). */
typedef struct {
  int64_t n_slabs;
  int64_t capacity;       /* total particle slots */
  int64_t off_z, off_mu, off_E, off_uid, off_flags, off_ev;  /* SoA arrays [capacity] */
  int64_t off_slab_base, off_slab_cap, off_slab_tail, off_slab_dead, off_slab_inst;
  int64_t off_dens, off_cur, off_counters;
  int64_t dens_len, cur_len;  /* elements of the int bins (u64 / i64) */
  int32_t state_bytes;        /* 4 (binary32) or 8 (binary64) for z and mu */
  int32_t flags_spin_shift, flags_layer_shift, flags_layer_bits, flags_gen_shift;
  uint32_t flags_dead_bit;
  int64_t off_w;              /* uint32 weights [capacity] in 2^-16 units, or -1 */
} pic_layout;

typedef struct pic_ctx pic_ctx;

/* Bytes of device workspace a context for `cfg` needs.  PIC_EINVAL on a bad config. */
pic_status pic_workspace_size(const pic_config* cfg, int64_t* bytes);

/* Set up one simulation of the 1-D hot-electron Boltzmann equation, Eq. (9), by the
 * particle-in-cell method of Sec. III.A for the layer stacks and parameters in `cfg`
 * (Eqs. 2, 7, 8, 19): validate `cfg` (PIC_EINVAL), lay out the caller's workspace
 * (PIC_ENOMEM if smaller than pic_workspace_size()), upload the tables and clear the
 * particles, bins and counters.  `stream` is a hipStream_t (or NULL).  The context is
 * host memory owned by the library until pic_destroy(). */
pic_status pic_init(const pic_config* cfg, void* workspace, int64_t workspace_bytes,
                    void* stream, pic_ctx** out);

/* Set the source schedule, Eq. (17): sched[i*n_steps + n] primaries of instance i are
 * created at the start of step n (host array; each row must sum to n_primaries). */
pic_status pic_inject(pic_ctx* ctx, const int64_t* sched);

/* Bytes of the static workspace behind pic_init_static(), one array per device. */
#define PIC_STATIC_WORKSPACE_BYTES (64ll << 20)

/* Allocation-free set-up, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): pic_init() with
 * the library's own static device array of PIC_STATIC_WORKSPACE_BYTES on the current
 * device as the workspace, so that neither this call nor the context's later calls
 * allocate device memory.  Every other call works on the context as on any other;
 * pic_deposit() and pic_backward() still write to caller-owned device arrays.  The
 * context launches its steps directly (pic_tuning.use_graph = 0; setting it to 1 makes
 * pic_step() instantiate a graph, which may allocate).  Each device holds its array from
 * the library's first use on that device until the process ends, and the array keeps the
 * previous context's contents (the set-up clears what must start at zero).  One live
 * context per device may own the array: a second call on the same device before
 * pic_destroy() of the first returns PIC_ESTATE (two contexts sharing it would race).
 * PIC_ENOMEM if the problem's workspace (pic_workspace_size) exceeds
 * PIC_STATIC_WORKSPACE_BYTES.  `stream` must belong to the current device. */
pic_status pic_init_static(const pic_config* cfg, void* stream, pic_ctx** out);

/* Enqueue n time steps (the next ones after those already run).  One step is the Strang
 * splitting of Eq. (15) for every superparticle of every instance: Source(dt/2) (the
 * primaries of the schedule, Eq. 17), Transport(dt/2) (Eq. 18 with vacuum reflection and
 * the stochastic interfaces of Sec. III.A), Scattering(dt) (one Monte-Carlo event with
 * p = 1 - exp(-dt/tau_eff), Eq. 2: elastic, Eq. 8, or inelastic with a secondary, Eqs. 6,
 * 7, 19; products below E_min removed), Transport(dt/2), then the moments of Eqs. (16)
 * and (23) added to the integer bins of the step.  One kernel launch per
 * pic_tuning.sub_steps steps.  PIC_EINVAL if the steps would go beyond n_steps,
 * PIC_ESTATE before pic_inject().  Device conditions are reported by pic_counters(). */
pic_status pic_step(pic_ctx* ctx, int32_t n);

/* Enqueue one compaction pass now (slabs whose dead slots exceed
 * pic_tuning.compact_frac of their tail are compacted in place).  pic_step() already
 * runs it every compact_every steps; this entry lets a caller time it separately. */
pic_status pic_compact(pic_ctx* ctx);

/* The moments of the run so far as binary64: the density of Eq. (16) (carriers per depth
 * bin, energy bin and spin) and the spin-resolved current moment of Eq. (23) (sum of
 * v cos(theta) per depth bin and spin; j_s is the up minus the down column, units
 * dropped as in the paper).  Converts the integer bins: dens_out
 * [sum_i n_dslots*nz_i*NE*2] particle counts and cur_out [sum_i n_cslots*nz_i*2] in
 * nm/fs; instances are concatenated in order.  With PIC_F_WEIGHTS both are weighted sums (the integer density
 * bins hold weights in 2^-16 units, the current bins rint(v cos(theta) w 2^32) per
 * carrier).  Device pointers (either may be NULL).  Enqueued, async. */
pic_status pic_deposit(pic_ctx* ctx, double* dens_out, double* cur_out);

/* Generation moment (context created with PIC_F_GEN_MOMENT): the sum of the generation
 * labels (1: primary, each secondary its parent's + 1, capped at 255) of the carriers
 * deposited in each density cell, per (density slot, depth, spin): gen_out
 * [sum_i n_dslots*nz_i*2], binary64 (exact integers), instances concatenated; divided by
 * the energy-summed density it is the mean generation map of Sec. V.  With
 * PIC_F_WEIGHTS the labels are weighted (sum of w * label, w in units of 1).  Device pointer.
 * Enqueued, async.  PIC_ESTATE without the flag. */
pic_status pic_generations(pic_ctx* ctx, double* gen_out);

/* Likelihood-ratio adjoint of the run (score-function estimator over the Monte-Carlo
 * decisions of Sec. III.A: the event probability of Eq. 2, the channel choice of Eqs. 5
 * and 8, the interface transmissions): gradient of sum(g_dens*dens) + sum(g_cur*cur)
 * with respect to ln tau0 per channel and every transmission-table entry, written to
 * grad_out
 * (device, [n_channels + n_ttables*t_entries], summed over instances).  Replays the run
 * from step 0 with the same random streams (the particle state is rebuilt; bins are
 * untouched).  estimator 0: causal score carried by each carrier (needs K <= 16 and
 * adjoint 1 or 3); 1: whole-tree return, two replays (adjoint 2 or 3).  g_dens / g_cur:
 * device arrays laid out like pic_deposit's outputs (either may be NULL).  Parameter
 * order: ln tau0 of channels 0..n_channels-1, then T[t][e] row-major.  The result is an
 * unbiased Monte-Carlo estimate on the same random streams as the forward run.  The
 * replay advances one step per launch in workgroups of at most 256 threads (the grid
 * scaled to keep the tuning's number of waves), writes z back every min(z_every, 4) steps
 * and compacts every min(compact_every, 8) steps (compact_every 0: never) the slabs whose
 * dead slots exceed max(compact_frac, 0.1) of their tail, moving score rows (causal) and
 * partial returns (whole-tree) with their carriers.  Synchronizes. */
pic_status pic_backward(pic_ctx* ctx, const double* g_dens, const double* g_cur,
                        double* grad_out, int32_t estimator);

/* Synchronize and copy the per-step counters to host_out [n_steps][PIC_NCOUNTERS]
 * (may be NULL).  Reports asynchronous device conditions. */
pic_status pic_counters(pic_ctx* ctx, int64_t* host_out);

/* Clear particles, bins and counters and rewind to step 0 (schedule is kept). */
pic_status pic_reset(pic_ctx* ctx);

pic_status pic_set_tuning(pic_ctx* ctx, const pic_tuning* t);
pic_status pic_get_tuning(const pic_ctx* ctx, pic_tuning* t);
pic_status pic_layout_of(const pic_ctx* ctx, pic_layout* out);

/* Time candidate tunings and store the fastest in the context (and in a per-device cache
 * keyed by the config signature): workgroup size and grid on the first `trial_steps`
 * steps of this context's run, then the compaction cadence and the z write-back period
 * on the first 4 x trial_steps.  Resets the context before and after.  Synchronizes. */
pic_status pic_autotune(pic_ctx* ctx, int32_t trial_steps, pic_tuning* best);

/* Per-launch timing, for measurement.  pic_time_kernels(ctx, 1) makes the following
 * pic_step calls launch directly (no graph) and record HIP events around each step-kernel
 * launch and its compaction; pic_time_kernels(ctx, 0) stops.  Either call synchronizes
 * and drops the events recorded so far. */
pic_status pic_time_kernels(pic_ctx* ctx, int32_t enable);

/* Synchronize and report the launches timed since timing was enabled: out[k*6 + 0..5] =
 * milliseconds of the step launch, of the compaction after it (about 0 when none ran),
 * the carrier-steps that took the common path (no boundary, certainly no event) and
 * the ones that took the general path, the launch's first step and its number of steps
 * (host array, up to max_steps rows; *n_out = launches recorded).  The recorded events
 * are dropped, except when out is NULL: then only *n_out is set. */
pic_status pic_kernel_times(pic_ctx* ctx, double* out, int32_t max_steps, int32_t* n_out);

void pic_destroy(pic_ctx* ctx);
const char* pic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
