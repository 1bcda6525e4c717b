// Internal layout shared by the device kernels and the host side of libpic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic.h"

namespace pic {

constexpr int kMaxL = PIC_MAX_LAYERS;
constexpr int kMaxT = PIC_MAX_TTABLES * PIC_MAX_TENTRIES;
constexpr int kMaxHits = 8;
constexpr int kMaxK = PIC_MAX_CHANNELS + PIC_MAX_TTABLES * PIC_MAX_TENTRIES;  // adjoint parameters
constexpr int kMaxCausalK = 16;
constexpr int kNC = PIC_NCOUNTERS;

// Random-number purposes (fourth counter word).  One fixed slot per purpose so that a
// branch taken or not taken never shifts the draws of another decision.
constexpr uint32_t kTagScat = 0x000u;    // words: (unused), channel, new direction, split
constexpr uint32_t kTagSpawn = 0x100u;   // words: direction, spin, lineage, lineage fallback
constexpr uint32_t kTagHalf1 = 0x200u;   // + i: i-th interface draw of the first half step
constexpr uint32_t kTagHalf2 = 0x300u;   // + i: same for the second half step
constexpr uint32_t kTagInject = 0x400u;  // counter (root, 0, ~0, tag): depth, dir, spin, E
constexpr uint32_t kTagDecide = 0x500u;  // counter (lo, hi, 2m, tag): event decisions of
                                         // steps 2m (word 0) and 2m + 1 (word 1)

// Packed per-particle flags.
constexpr uint32_t kSpinMask = 1u;
constexpr int kLayerShift = 1;
constexpr uint32_t kLayerMask = 0xFu;
constexpr int kGenShift = 8;
constexpr uint32_t kGenMask = 0xFFu;
constexpr uint32_t kDead = 0x80000000u;
// Steps since the stored z was written, counted from the last write-back boundary (see
// StepArgs::z_phase); 0 outside a pic_step call.
constexpr int kStampShift = 5;
constexpr uint32_t kStampMask = 0x7u;
constexpr int kMaxZEvery = 8;
// Steps one launch of the step kernel may advance.
constexpr int kMaxSub = 2;
// Adjoint replays: the first step whose non-event score term of a carrier is still pending
// lives in flag bits 16-30 (the forward never sets them).
constexpr int kNfShift = 16;
constexpr uint32_t kNfMask = 0x7FFFu;
__host__ __device__ __forceinline__ uint32_t nf_of(uint32_t fl) { return (fl >> kNfShift) & kNfMask; }
__host__ __device__ __forceinline__ uint32_t with_nf(uint32_t fl, uint32_t nf) {
  return (fl & ~(kNfMask << kNfShift)) | (nf << kNfShift);
}

// Energy-bin lookup table: one entry per bucket of 2^22 energy units (the top 10 bits).
constexpr int kEBucketShift = 22;
constexpr int kEBuckets = 1 << (32 - kEBucketShift);

// Device status bits.
constexpr uint32_t kStOverflow = 1u;
constexpr uint32_t kStHits = 2u;

// Per-instance tables as the kernels read them (copied into LDS per workgroup).
struct alignas(32) DevInst {
  double4 lay[kMaxL];          // (z_lo, z_hi, 1/tau_el, P(up) of a secondary)
  double2 chan[kMaxL][2];      // per (layer, spin): (speed, 1/tau0)
  double ratio[kMaxL][2][2];   // per (layer, spin, direction +z/-z): v_next / v_this
  double T_scale, inv_dz;
  double src_lo, src_hi, src_lambda, src_cd, src_up;
  double e_scale;              // energy tables: nodes at E = k / e_scale eV
  double w_scale;              // weight table: nodes at E = k / w_scale eV
  uint32_t e_lo[2], e_span[2];
  int32_t n_layers, t_entries, nz, n_slabs;
  uint64_t root_offset;
  int64_t dens_off, cur_off;   // element offsets of this instance in the global bins
  int64_t gen_off;             // ... in the generation-moment bins
  int64_t etab_off;            // ... in the energy tables ([v rows | rate rows][channel][node])
  int32_t slab0, e_nodes;      // e_nodes = 0: constant speeds and rates
  int32_t w_nodes, pad1;       // weight table nodes per spin (0: weight 1); rows [2][w_nodes]
                               // follow the energy tables at etab_off + 2 n_ch e_nodes
  uint8_t tt[kMaxL - 1][2][2]; // transmission table per (interface, direction, spin)
  uint8_t chi[kMaxL][2];       // channel index per (layer, spin) (adjoint parameter slot)
  uint8_t n_ch;                // channels (rows of each energy table)
  uint8_t pad2[3];
  double T[kMaxT];             // [table][entry]; only the first n_ttables*t_entries used
};
// bytes of DevInst that precede the transmission tables
constexpr int kInstHead = (int)offsetof(DevInst, T);
static_assert(kInstHead % 16 == 0, "the head is copied in 16-byte words");

struct StepArgs {
  void* z;
  void* mu;
  uint32_t* E;
  uint64_t* uid;
  uint32_t* flags;
  uint64_t* ev;                // per-particle event counts (debug) or null
  const int64_t* slab_base;
  const int32_t* slab_cap;
  int32_t* slab_tail;
  int32_t* slab_dead;
  const int32_t* slab_inst;
  const int32_t* slab_k;
  const DevInst* inst;
  const int64_t* inj_cum;      // [n_inst][n_steps + 1] cumulative primaries per step
  const uint32_t* e_edges;
  const uint8_t* e_bucket;     // [1024] bin of the lower end of each 2^22 energy bucket
  uint64_t* dens;
  int64_t* cur;
  int64_t* counters;           // [n_steps][kNC]
  int32_t* queue;              // [n_steps] slab dispenser
  uint32_t* status;
  unsigned long long* stats;   // [n_steps][2] carriers finished by the common step / left
  int32_t n_slabs, n_inst, n_ebins, n_steps;
  int32_t step;
  uint32_t key0, key1;
  uint32_t e_min;
  double dt, h;
  int32_t tau_exp2, secondaries, debug;
  int32_t absorb_next;         // below E_min: removed at the next event (else at once)
  int32_t dens_on, cur_on;     // this step deposits density / current
  int32_t dens_slot, cur_slot;
  int32_t dens_lds;            // density privatised in LDS (else global atomics)
  int32_t lds_dens_words;      // bins of the LDS density histogram
  int32_t dens16;              // LDS density slices hold 16-bit counters, two per word
                               // (unweighted runs without energy tables)
  int32_t lds_cur_words;       // u64 words of the LDS current histogram
  int32_t inst_bytes;          // bytes of DevInst copied into LDS
  // Write-back schedule of z on the common path: the stored z of a carrier is its
  // position at the start of step (this step - z_phase + stamp); the steps in between
  // were straight flights and are recomputed.  z_write: this step stores z and clears
  // the stamps (the last step of a write-back period or of a pic_step call).
  int32_t z_phase, z_write;
  // The steps step .. step + n_sub - 1 that one launch of the step kernel advances
  // (sub-step j = step + j), and the byte offsets of their LDS histogram slices (-1: the
  // sub-step deposits no such moment) and of the per-wave queues.
  int32_t n_sub;
  int32_t sub_dens_on[kMaxSub], sub_cur_on[kMaxSub];
  int32_t sub_dens_slot[kMaxSub], sub_cur_slot[kMaxSub];
  int32_t sub_z_phase[kMaxSub], sub_z_write[kMaxSub];
  int32_t lds_dens_at[kMaxSub], lds_cur_at[kMaxSub];
  int32_t lds_q_at, lds_q_bytes;
  // generation moment: sum of generation labels per (density slot, z, spin), taken with
  // the density (LDS slice per sub-step at lds_gen_at, u32), or null
  uint64_t* gen;
  int32_t lds_gen_at[kMaxSub];
  // energy tables of all instances (binary64, at DevInst::etab_off), or null; copied per
  // instance into dynamic LDS at lds_etab_at (step kernel; etab_words doubles at most)
  const double* etab;
  int32_t lds_etab_at, etab_words;
  // superparticle weights (2^-16 units) per slot, or null: the moments are plain counts
  uint32_t* wt;
  // per-wave copies of the state of the carriers in the sub-step-0 queue (stage_wave_bytes
  // per wave), so that their general pass reads LDS instead of HBM; -1: not staged
  int32_t lds_stage_at;
  // per-wave copies of the state of the first kStage1 entries of the sub-step-1 queue
  // (stage1_wave_bytes per wave); -1: not staged
  int32_t lds_stage1_at;
  // The two passes of the whole-tree adjoint run by the step kernel itself (modes
  // kModeRet, kModeScore of pic_kernels.hip), with the forward's launch structure:
  // per-slot partial returns, per-root returns, dL/d(density), dL/d(current) (pass 1
  // copies the launch's slices into LDS at lds_cur_at), the gradient and its length, and
  // the LDS gradient accumulator of pass 2 (doubles [adj_K] at lds_grad_at).
  double* adj_r;
  double* adj_R;
  const double* adj_gd;
  const double* adj_gc;
  double* adj_grad;
  int32_t adj_pass;            // 0: forward; 1, 2: the whole-tree adjoint's passes
  int32_t adj_K, lds_grad_at;
};

struct AdjArgs {
  StepArgs s;                  // the dynamics, exactly as in the forward step
  double* S;                   // causal score rows [capacity][K]
  double* r;                   // per-carrier partial return [capacity]
  double* R;                   // per-tree return [n_roots]
  const double* g_dens;        // dL/d(density), laid out like the bins, or null
  const double* g_cur;         // dL/d(current) per nm/fs, or null
  double* grad;                // [K] accumulator
  int32_t K, n_ch;
};

struct CompactArgs {
  void* z;
  void* mu;
  uint32_t* E;
  uint64_t* uid;
  uint32_t* flags;
  uint64_t* ev;
  const int64_t* slab_base;
  int32_t* slab_tail;
  int32_t* slab_dead;
  int32_t n_slabs;
  float frac;
  double* S;                   // adjoint score rows [capacity][K] moved along, or null
  int32_t K;
  double* r;                   // adjoint partial returns moved along, or null
  uint32_t* w;                 // superparticle weights moved along, or null
};

// bytes of one wave's newborn queue (step kernel) and general-path slot queue (adjoint
// replay) in dynamic LDS
constexpr size_t kChildQueueBytes = 64 * (8 + 4 * 5);
constexpr size_t kSlowQueueBytes = 128 * 4;
// bytes of one wave's queues in the step kernel: newborns, then the slot queues of
// sub-step 0 (128 entries) and, in two-step launches, of sub-step 1 (256 entries)
constexpr size_t step_queue_bytes(int n_sub) {
  return kChildQueueBytes + 128 * 4 + (n_sub > 1 ? 256 * 4 : 0);
}

// bytes per wave of the staged sub-step-0 queue: z and cos(theta) (binary32 or binary64),
// E, flags and uid of each of its 128 entries
constexpr size_t stage_wave_bytes(bool fp64) { return 128 * ((fp64 ? 16 : 8) + 16); }
// the same for the first kStage1 entries of the sub-step-1 queue (two-step launches)
constexpr int kStage1 = 64;
constexpr size_t stage1_wave_bytes(bool fp64) { return kStage1 * ((fp64 ? 16 : 8) + 16); }

// Launch shape of one step.
struct StepLaunch {
  int grid, block;
  size_t lds;                  // dynamic LDS (histograms + per-wave queues)
  hipEvent_t ev[2];            // optional: recorded before and after the launch
};

// launchers (pic_kernels.hip)
hipError_t launch_step(const StepArgs& a, bool fp64, const StepLaunch& L, hipStream_t s);
hipError_t launch_compact(const CompactArgs& a, bool fp64, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& A, bool fp64, int adj, int grid, int block,
                          hipStream_t s);
hipError_t launch_adjoint_final(const AdjArgs& A, bool fp64, int adj, uint32_t n_steps,
                                hipStream_t s);
size_t step_static_lds();
hipError_t set_step_lds_limit(size_t bytes);
hipError_t launch_fill32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_convert(const uint64_t* dens, int64_t nd, const int64_t* cur, int64_t nc,
                          double* dout, double* cout, double dscale, hipStream_t s);

}  // namespace pic
