// Host side of the libpic C ABI: validation, workspace layout, table upload, the step
// driver (direct launches or a captured hipGraph) and the integer-to-binary64 bins.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pic_internal.h"

using namespace pic;

namespace {

thread_local std::string g_err;

pic_status fail(pic_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(PIC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

bool on_grid(double z) {
  const double q = z * 64.0;
  return std::isfinite(q) && q == std::floor(q) && std::fabs(q) < 9.0e15;
}

struct Plan {
  std::vector<int32_t> slab_inst, slab_k, slab_cap;
  std::vector<int64_t> slab_base;
  std::vector<int32_t> n_slabs_of, slab0_of;
  std::vector<int64_t> dens_off, cur_off, gen_off, etab_off;
  int64_t capacity = 0, dens_len = 0, cur_len = 0, gen_len = 0;
  int64_t etab_len = 0;        // doubles of all energy tables
  int etab_max = 0;            // doubles of the largest instance's tables
  int n_dslots = 0, n_cslots = 0, state_bytes = 4;
  bool debug = false;
  // byte offsets inside the workspace
  int64_t off_z, off_mu, off_E, off_uid, off_flags, off_ev;
  int64_t off_slab_base, off_slab_cap, off_slab_tail, off_slab_dead, off_slab_inst, off_slab_k;
  int64_t off_inst, off_inj, off_edges, off_dens, off_cur, off_counters, off_queue, off_status;
  int64_t off_stats, off_gen = -1, off_etab = -1, off_w = -1;
  int64_t off_grad = -1, off_S = -1, off_r = -1, off_R = -1;
  int K = 0;
  int64_t n_roots = 0;
  int64_t bytes = 0;
};

pic_status validate(const pic_config* c) {
  if (!c) return fail(PIC_EINVAL, "null config");
  if (c->n_instances < 1 || !c->inst) return fail(PIC_EINVAL, "need at least one instance");
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return fail(PIC_EINVAL, "dt must be > 0");
  if (c->n_steps < 1) return fail(PIC_EINVAL, "n_steps must be >= 1");
  if (c->tau_exp != 0 && c->tau_exp != 2) return fail(PIC_EINVAL, "tau_exp must be 0 or 2");
  if (c->n_ebins < 1 || c->n_ebins > PIC_MAX_EBINS) return fail(PIC_EINVAL, "bad n_ebins");
  for (int k = 1; k < c->n_ebins; ++k)
    if (!(c->e_edges[k] > c->e_edges[k - 1])) return fail(PIC_EINVAL, "energy edges must increase");
  if (c->dens_stride < 1 || c->cur_stride < 1) return fail(PIC_EINVAL, "strides must be >= 1");
  if (c->slab_primaries < 0) return fail(PIC_EINVAL, "slab_primaries must be >= 0");
  if (c->capacity_factor < 0 || !std::isfinite(c->capacity_factor))
    return fail(PIC_EINVAL, "capacity_factor must be >= 0");
  std::vector<std::pair<uint64_t, uint64_t>> roots;  // [root_offset, + n_primaries) per instance
  for (int i = 0; i < c->n_instances; ++i) {
    const pic_instance& I = c->inst[i];
    const std::string w = "instance " + std::to_string(i) + ": ";
    if (I.n_layers < 1 || I.n_layers > PIC_MAX_LAYERS) return fail(PIC_EINVAL, w + "bad n_layers");
    if (I.n_channels < 1 || I.n_channels > PIC_MAX_CHANNELS) return fail(PIC_EINVAL, w + "bad n_channels");
    if (I.n_ttables < 1 || I.n_ttables > PIC_MAX_TTABLES) return fail(PIC_EINVAL, w + "bad n_ttables");
    if (I.t_entries < 1 || I.t_entries > PIC_MAX_TENTRIES) return fail(PIC_EINVAL, w + "bad t_entries");
    for (int l = 0; l <= I.n_layers; ++l)
      if (!on_grid(I.z_bound[l])) return fail(PIC_EINVAL, w + "z_bound must lie on the 2^-6 nm grid");
    for (int l = 0; l < I.n_layers; ++l) {
      if (!(I.z_bound[l + 1] > I.z_bound[l])) return fail(PIC_EINVAL, w + "z_bound must increase");
      for (int s = 0; s < 2; ++s)
        if (I.ch_of[l][s] < 0 || I.ch_of[l][s] >= I.n_channels) return fail(PIC_EINVAL, w + "bad ch_of");
      if (!(I.inv_tau_el[l] >= 0.0) || !std::isfinite(I.inv_tau_el[l])) return fail(PIC_EINVAL, w + "bad inv_tau_el");
      if (!(I.P0[l] >= -1.0 && I.P0[l] <= 1.0)) return fail(PIC_EINVAL, w + "P0 outside [-1,1]");
    }
    for (int k = 0; k < I.n_layers - 1; ++k)
      for (int d = 0; d < 2; ++d)
        for (int s = 0; s < 2; ++s)
          if (I.tt_of[k][d][s] < 0 || I.tt_of[k][d][s] >= I.n_ttables) return fail(PIC_EINVAL, w + "bad tt_of");
    if (I.e_nodes != 0 && (I.e_nodes < 2 || I.e_nodes > PIC_MAX_TENTRIES))
      return fail(PIC_EINVAL, w + "e_nodes must be 0 or 2..PIC_MAX_TENTRIES");
    // energies are below 4 eV: the node index (E e_scale) must fit an int
    if (I.e_nodes && (!(I.e_scale > 0.0) || !(I.e_scale <= 1e8)))
      return fail(PIC_EINVAL, w + "e_scale must be in (0, 1e8]");
    for (int ch = 0; ch < I.n_channels; ++ch) {
      if (!I.e_nodes && (!(I.v[ch] > 0.0) || !std::isfinite(I.v[ch])))
        return fail(PIC_EINVAL, w + "speeds must be > 0");
      if (!(I.inv_tau0[ch] >= 0.0) || !std::isfinite(I.inv_tau0[ch])) return fail(PIC_EINVAL, w + "inv_tau0 must be >= 0");
      for (int k = 0; k < I.e_nodes; ++k) {
        if (!(I.v_node[ch][k] > 0.0) || !std::isfinite(I.v_node[ch][k]))
          return fail(PIC_EINVAL, w + "tabled speeds must be > 0");
        if (!(I.r_node[ch][k] >= 0.0) || !std::isfinite(I.r_node[ch][k]))
          return fail(PIC_EINVAL, w + "tabled rates must be >= 0");
      }
    }
    for (int t = 0; t < I.n_ttables; ++t)
      for (int e = 0; e < I.t_entries; ++e)
        if (!(I.T[t][e] >= 0.0 && I.T[t][e] <= 1.0)) return fail(PIC_EINVAL, w + "T outside [0,1]");
    if (c->flags & PIC_F_WEIGHTS) {
      if (I.w_nodes < 0 || I.w_nodes > PIC_MAX_TENTRIES)
        return fail(PIC_EINVAL, w + "w_nodes must be 0..PIC_MAX_TENTRIES");
      if (I.w_nodes && !(I.w_scale >= 0.0 && I.w_scale <= 1e8))
        return fail(PIC_EINVAL, w + "w_scale must be in [0, 1e8]");
      for (int s = 0; s < 2; ++s)
        for (int k = 0; k < I.w_nodes; ++k)
          if (!(I.w_node[s][k] >= 0x1p-16 && I.w_node[s][k] <= 0x1p15))
            return fail(PIC_EINVAL, w + "weights must be in [2^-16, 2^15]");
    }
    if (I.t_entries > 1 && (!(I.T_scale > 0.0) || !(I.T_scale <= 1e8)))
      return fail(PIC_EINVAL, w + "T_scale must be in (0, 1e8]");
    if (!(I.src_z_lo >= I.z_bound[0] && I.src_z_hi <= I.z_bound[I.n_layers] && I.src_z_lo <= I.src_z_hi))
      return fail(PIC_EINVAL, w + "source region outside the stack");
    if (!(I.src_lambda >= 0.0) || !std::isfinite(I.src_lambda)) return fail(PIC_EINVAL, w + "bad src_lambda");
    if (I.src_lambda > 0.0 && !(I.src_cd > 0.0 && I.src_cd <= 1.0)) return fail(PIC_EINVAL, w + "bad src_cd");
    if (!(I.src_up_frac >= 0.0 && I.src_up_frac <= 1.0)) return fail(PIC_EINVAL, w + "bad src_up_frac");
    for (int s = 0; s < 2; ++s)
      if ((uint64_t)I.src_e_lo[s] + I.src_e_span[s] > 0xFFFFFFFFull) return fail(PIC_EINVAL, w + "energy range overflows");
    if (I.nz < 1 || !(I.inv_dz > 0.0) || !std::isfinite(I.inv_dz)) return fail(PIC_EINVAL, w + "bad depth bins");
    if (I.n_primaries < 0) return fail(PIC_EINVAL, w + "n_primaries < 0");
    if (I.root_offset + (uint64_t)I.n_primaries > 0x100000000ull)
      return fail(PIC_EINVAL, w + "root ids must fit in 32 bits");
    if (I.n_primaries > 0) roots.emplace_back(I.root_offset, I.root_offset + (uint64_t)I.n_primaries);
  }
  // Root ids key the random streams of a primary tree (and its slot of per-tree returns in
  // the adjoint): two instances sharing a root would replay each other's trees.
  std::sort(roots.begin(), roots.end());
  for (size_t k = 1; k < roots.size(); ++k)
    if (roots[k].first < roots[k - 1].second)
      return fail(PIC_EINVAL, "instances have overlapping root id ranges [root_offset, root_offset + n_primaries)");
  if (c->adjoint < 0 || c->adjoint > 3) return fail(PIC_EINVAL, "adjoint must be 0..3");
  if (c->adjoint) {
    const pic_instance& I0 = c->inst[0];
    for (int i = 1; i < c->n_instances; ++i)
      if (c->inst[i].n_channels != I0.n_channels || c->inst[i].n_ttables != I0.n_ttables ||
          c->inst[i].t_entries != I0.t_entries)
        return fail(PIC_EINVAL, "adjoint needs the same table shapes in every instance");
    if (c->n_steps > 32767) return fail(PIC_EINVAL, "adjoint supports at most 32767 steps");
    const int K = I0.n_channels + I0.n_ttables * I0.t_entries;
    if ((c->adjoint & 1) && K > kMaxCausalK)
      return fail(PIC_EINVAL, "causal adjoint supports at most 16 parameters");
  }
  return PIC_OK;
}

double default_capacity(const pic_config* c, const pic_instance& I) {
  if (c->capacity_factor > 0) return c->capacity_factor;
  if (!(c->flags & PIC_F_SECONDARIES)) return 1.0;
  if (c->e_min_fx == 0) return 32.0;
  const uint64_t e0 = std::max((uint64_t)I.src_e_lo[0] + I.src_e_span[0],
                               (uint64_t)I.src_e_lo[1] + I.src_e_span[1]);
  // every carrier of a tree keeps at least E_min, and energy is conserved; with removal
  // at the next event carriers below E_min live on as well: twice the headroom
  const double f = (double)(e0 / c->e_min_fx) + 2.0;
  return std::min<double>((c->flags & PIC_F_ABSORB_NEXT) ? 2.0 * f : f, 64.0);
}

// Workgroups of the step kernel's default launch shape that run at once on the device
// (two 512-thread workgroups per CU).
int64_t resident_step_workgroups() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return 2 * (int64_t)cus;
}

// Default primaries per slab.  Instances of equal size give slabs of about equal work: their
// slab count is then a multiple of the workgroups that run at once (twice that where the
// adjoint uses the one-step replay, which runs four 256-thread workgroups per CU), so that each
// workgroup takes as many slabs as the others, with at most 32768 primaries per slab (one
// slab per workgroup where that suffices: the spin valve's launch measured 0.48 ms against
// 0.50 with two slabs per workgroup and 0.53 with four).  Otherwise 16384 primaries (fewer
// slab and instance switches per workgroup), smaller when the problem would give fewer
// than 2048 slabs, which the work-ordered slab queue balances over the workgroups.
int default_slab_primaries(const pic_config* c, int64_t total) {
  bool uniform = c->n_instances > 0;
  for (int i = 1; i < c->n_instances; ++i)
    uniform = uniform && c->inst[i].n_primaries == c->inst[0].n_primaries;
  // the one-step replay: the causal estimator, and the whole tree with energy tables,
  // weights or debug counts (otherwise the step kernel replays the whole tree)
  bool tables = false;
  for (int i = 0; i < c->n_instances; ++i) tables = tables || c->inst[i].e_nodes > 0;
  const bool replay = (c->adjoint & 1) ||
                      ((c->adjoint & 2) && (tables || (c->flags & (PIC_F_WEIGHTS | PIC_F_DEBUG))));
  const int64_t R = resident_step_workgroups() * (replay ? 2 : 1);
  if (uniform && R % c->n_instances == 0) {
    const int64_t k = std::max<int64_t>(1, (total + R * 32768 - 1) / (R * 32768));
    const int64_t S = R * k / c->n_instances;  // slabs per instance
    const int64_t N = c->inst[0].n_primaries;
    return (int)std::max<int64_t>(256, (N + S - 1) / S);
  }
  return (int)std::min<int64_t>(16384, std::max<int64_t>(256, (total + 2047) / 2048));
}

Plan make_plan(const pic_config* c) {
  Plan p;
  p.state_bytes = (c->flags & PIC_F_STATE_FP64) ? 8 : 4;
  p.debug = (c->flags & PIC_F_DEBUG) != 0;
  int64_t total = 0;
  for (int i = 0; i < c->n_instances; ++i) total += c->inst[i].n_primaries;
  const int P = c->slab_primaries > 0 ? c->slab_primaries : default_slab_primaries(c, total);
  p.n_dslots = (c->n_steps + c->dens_stride - 1) / c->dens_stride;
  p.n_cslots = (c->n_steps + c->cur_stride - 1) / c->cur_stride;
  // Slabs are handed out in the order of the slab table, so the instances are laid out
  // by decreasing expected work per slab (primaries per slab times the mean pump energy,
  // to which the size of a cascade is proportional): the last slabs of a launch are then
  // the lightest and the workgroups run out of work at nearly the same time.  Each
  // instance's slabs stay contiguous, and no result depends on this order.
  std::vector<int> order(c->n_instances);
  std::vector<double> work(c->n_instances);
  for (int i = 0; i < c->n_instances; ++i) {
    const pic_instance& I = c->inst[i];
    const int64_t S = std::max<int64_t>(1, (I.n_primaries + P - 1) / P);
    const double per = (double)((I.n_primaries + S - 1) / S);
    const double up = std::min(1.0, std::max(0.0, I.src_up_frac));
    const double e0 = up * ((double)I.src_e_lo[0] + 0.5 * I.src_e_span[0]) +
                      (1.0 - up) * ((double)I.src_e_lo[1] + 0.5 * I.src_e_span[1]);
    order[i] = i;
    work[i] = per * e0;
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  p.n_slabs_of.assign(c->n_instances, 0);
  p.slab0_of.assign(c->n_instances, 0);
  for (const int i : order) {
    const pic_instance& I = c->inst[i];
    const int64_t N = I.n_primaries;
    const int64_t S = std::max<int64_t>(1, (N + P - 1) / P);
    const int64_t per = (N + S - 1) / S;
    const double f = default_capacity(c, I);
    int64_t cap = (int64_t)std::ceil((double)per * f) + 64;
    cap = (cap + 63) & ~int64_t(63);
    if (cap > (int64_t)1 << 28) cap = (int64_t)1 << 28;  // 32-bit byte offsets inside a slab
    p.n_slabs_of[i] = (int32_t)S;
    p.slab0_of[i] = (int32_t)p.slab_inst.size();
    for (int64_t k = 0; k < S; ++k) {
      p.slab_inst.push_back(i);
      p.slab_k.push_back((int32_t)k);
      p.slab_cap.push_back((int32_t)cap);
      p.slab_base.push_back(p.capacity);
      p.capacity += cap;
    }
  }
  for (int i = 0; i < c->n_instances; ++i) {
    const pic_instance& I = c->inst[i];
    p.dens_off.push_back(p.dens_len);
    p.cur_off.push_back(p.cur_len);
    p.gen_off.push_back(p.gen_len);
    p.etab_off.push_back(p.etab_len);
    const int et_words = 2 * I.n_channels * I.e_nodes;
    // weight rows [2][w_nodes] follow the instance's energy tables (read at injection)
    const int w_words = (c->flags & PIC_F_WEIGHTS) ? 2 * I.w_nodes : 0;
    p.etab_len += et_words + w_words;
    p.etab_max = std::max(p.etab_max, et_words);
    p.dens_len += (int64_t)p.n_dslots * I.nz * c->n_ebins * 2;
    p.cur_len += (int64_t)p.n_cslots * I.nz * 2;
    if (c->flags & PIC_F_GEN_MOMENT) p.gen_len += (int64_t)p.n_dslots * I.nz * 2;
  }
  const int64_t C = p.capacity, NS = (int64_t)p.slab_inst.size(), NI = c->n_instances;
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o = align256(o + bytes);
    return at;
  };
  p.off_z = take(C * p.state_bytes);
  p.off_mu = take(C * p.state_bytes);
  p.off_E = take(C * 4);
  p.off_uid = take(C * 8);
  p.off_flags = take(C * 4);
  p.off_ev = p.debug ? take(C * 8) : -1;
  p.off_slab_base = take(NS * 8);
  p.off_slab_cap = take(NS * 4);
  p.off_slab_tail = take(NS * 4);
  p.off_slab_dead = take(NS * 4);
  p.off_slab_inst = take(NS * 4);
  p.off_slab_k = take(NS * 4);
  p.off_inst = take(NI * (int64_t)sizeof(DevInst));
  p.off_inj = take(NI * ((int64_t)c->n_steps + 1) * 8);
  p.off_edges = take(PIC_MAX_EBINS * 4 + kEBuckets);  // edges, then the bucket table
  p.off_dens = take(p.dens_len * 8);
  p.off_cur = take(p.cur_len * 8);
  p.off_counters = take((int64_t)c->n_steps * kNC * 8);
  p.off_queue = take((int64_t)c->n_steps * 4 * 2);
  p.off_status = take(64);
  p.off_stats = take((int64_t)c->n_steps * 2 * 8);
  if (c->flags & PIC_F_GEN_MOMENT) p.off_gen = take(p.gen_len * 8);
  if (p.etab_len > 0) p.off_etab = take(p.etab_len * 8);
  if (c->flags & PIC_F_WEIGHTS) p.off_w = take(C * 4);
  if (c->adjoint) {
    const pic_instance& I0 = c->inst[0];
    p.K = I0.n_channels + I0.n_ttables * I0.t_entries;
    for (int i = 0; i < c->n_instances; ++i)
      p.n_roots = std::max<int64_t>(p.n_roots, (int64_t)c->inst[i].root_offset + c->inst[i].n_primaries);
    p.off_grad = take((int64_t)p.K * 8);
    if (c->adjoint & 1) p.off_S = take(C * p.K * 8);
    if (c->adjoint & 2) {
      p.off_r = take(C * 8);
      p.off_R = take(std::max<int64_t>(p.n_roots, 1) * 8);
    }
  }
  p.bytes = o;
  return p;
}

}  // namespace

struct pic_ctx {
  int static_dev = -1;         // >= 0: the workspace is that device's static array
  pic_config cfg;
  std::vector<pic_instance> inst;
  Plan plan;
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  std::vector<DevInst> h_inst;
  std::vector<double> h_etab;
  std::vector<uint8_t> h_ebkt;
  std::vector<int64_t> h_inj;
  std::vector<int64_t> h_counters;
  int step = 0;
  bool sched_set = false;
  pic_tuning tune;
  size_t lds_bytes = 0, max_lds = 0;
  int lds_dens_words = 0, lds_cur_words = 0, inst_bytes = 0;
  bool dens_lds = true;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int g_start = -1, g_n = -1;
  // per-launch timing: events before and after each step launch and after its compaction
  bool timing = false;
  std::vector<std::array<hipEvent_t, 3>> tev;
  std::vector<int> tstep, tnsub;

  template <typename T>
  T* at(int64_t off) const { return off < 0 ? nullptr : (T*)(ws + off); }
};

namespace {

void drop_events(pic_ctx* c) {
  for (auto& ev : c->tev)
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  c->tev.clear();
  c->tstep.clear();
  c->tnsub.clear();
}

void drop_graph(pic_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->g_start = c->g_n = -1;
}

// bytes per entry of the LDS density and generation slices: u64 sums of weights in a
// weighted run, u32 counts otherwise
size_t dens_elem(const pic_ctx* c) { return c->plan.off_w >= 0 ? 8 : 4; }

// LDS bytes per compute unit (160 KB on gfx950).
size_t lds_per_cu() {
  static size_t cached = 0;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (cached) return cached;
  int dev = 0, bytes = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      bytes > 0)
    cached = (size_t)bytes;
  else
    cached = 160 * 1024;
  return cached;
}

// LDS one workgroup of `block` threads may use without lowering the number of its
// workgroups per CU below the register limit (at most 16 waves of the step kernel per CU).
size_t lds_per_wg(int block) {
  return lds_per_cu() / (size_t)std::max(1, 16 / (block / 64));
}

// Dynamic LDS layout of one step launch over n_sub sub-steps: the density slices (of the
// sub-steps that deposit density, when density goes to LDS), the current slices, the
// per-wave queues, then (where they fit) the per-wave copies of the sub-step-0 queue's
// carrier state.  Fills the offsets in `a` (if given) and returns the bytes.
size_t step_layout(const pic_ctx* c, int block, int n_sub, const int* dens_on, const int* cur_on,
                   StepArgs* a, bool dens16 = false, int adj_pass = 0) {
  size_t off = 0;
  // a density slice: u64 weight sums, u32 counts, or 16-bit counts packed two per word
  const size_t dens_bytes = dens16 ? (size_t)c->lds_dens_words * 2
                                   : (size_t)c->lds_dens_words * dens_elem(c);
  // the adjoint passes deposit no moments: pass 1 keeps its dL/d(current) slices where
  // the current slices are, pass 2 its gradient accumulator
  for (int j = 0; j < kMaxSub; ++j) {
    const bool d = j < n_sub && dens_on[j] && c->dens_lds && adj_pass == 0;
    if (a) a->lds_dens_at[j] = d ? (int32_t)off : -1;
    if (d) off = (off + dens_bytes + 15) & ~(size_t)15;
  }
  if (a) a->dens16 = dens16 ? 1 : 0;
  for (int j = 0; j < kMaxSub; ++j) {
    const bool u = j < n_sub && cur_on[j] && adj_pass != 2;
    if (a) a->lds_cur_at[j] = u ? (int32_t)off : -1;
    if (u) off = (off + (size_t)c->lds_cur_words * 8 + 15) & ~(size_t)15;
  }
  if (a) a->lds_grad_at = adj_pass == 2 ? (int32_t)off : -1;
  if (adj_pass == 2) off = (off + (size_t)c->plan.K * 8 + 15) & ~(size_t)15;
  // generation-moment slices (u32 per (z, spin)) beside the density slices in LDS
  for (int j = 0; j < kMaxSub; ++j) {
    const bool g = j < n_sub && dens_on[j] && c->dens_lds && c->plan.off_gen >= 0 && adj_pass == 0;
    if (a) a->lds_gen_at[j] = g ? (int32_t)off : -1;
    if (g) off = (off + (size_t)c->lds_cur_words * dens_elem(c) + 15) & ~(size_t)15;
  }
  // the energy tables of the workgroup's instance
  if (a) a->lds_etab_at = c->plan.etab_max ? (int32_t)off : -1;
  off = (off + (size_t)c->plan.etab_max * 8 + 15) & ~(size_t)15;
  if (a) {
    a->lds_q_at = (int32_t)off;
    a->lds_q_bytes = (int32_t)step_queue_bytes(n_sub);
  }
  off += (size_t)(block / 64) * step_queue_bytes(n_sub);
  // copies of the sub-step-0 queue's carrier state, when they fit without costing a
  // workgroup per CU (at most 16 waves of the step kernel per CU, its register limit)
  const size_t stage_at = (off + 15) & ~(size_t)15;
  const size_t stage_end =
      stage_at + (size_t)(block / 64) * stage_wave_bytes(c->plan.state_bytes == 8);
  const size_t per_wg = lds_per_wg(block);
  const size_t stat = step_static_lds();
  const bool stage = stage_end + stat <= per_wg && stage_end <= c->max_lds;
  if (a) a->lds_stage_at = stage ? (int32_t)stage_at : -1;
  // and of the first entries of the sub-step-1 queue behind them (or in their place when
  // they do not fit), where those fit
  const size_t stage1_at = stage ? stage_end : stage_at;
  const size_t stage1_end =
      stage1_at + (size_t)(block / 64) * stage1_wave_bytes(c->plan.state_bytes == 8);
  const bool stage1 = n_sub > 1 && stage1_end + stat <= per_wg && stage1_end <= c->max_lds;
  if (a) a->lds_stage1_at = stage1 ? (int32_t)stage1_at : -1;
  return stage1 ? stage1_end : stage ? stage_end : off;
}

// LDS of a one-step launch that deposits both moments (the largest one-step layout).
size_t lds_for(const pic_ctx* c, int block) {
  const int on[kMaxSub] = {1, 1};
  return step_layout(c, block, 1, on, on, nullptr);
}

// Largest dynamic LDS a step launch may use: the device's per-workgroup limit minus the
// kernel's static LDS, after raising the kernels' dynamic-LDS attribute to it.
size_t device_lds_limit() {
  static size_t cached = 0;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (cached) return cached;
  int dev = 0, per_block = 65536;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  const size_t stat = step_static_lds();
  size_t lim = per_block > (int)stat ? (size_t)per_block - stat : 0;
  if (lim > 65536 - stat && set_step_lds_limit(lim) != hipSuccess) lim = 65536 - stat;
  cached = lim;
  return cached;
}

StepArgs step_args(const pic_ctx* c, int n) {
  const Plan& p = c->plan;
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.z = c->at<void>(p.off_z);
  a.mu = c->at<void>(p.off_mu);
  a.E = c->at<uint32_t>(p.off_E);
  a.uid = c->at<uint64_t>(p.off_uid);
  a.flags = c->at<uint32_t>(p.off_flags);
  a.ev = c->at<uint64_t>(p.off_ev);
  a.slab_base = c->at<int64_t>(p.off_slab_base);
  a.slab_cap = c->at<int32_t>(p.off_slab_cap);
  a.slab_tail = c->at<int32_t>(p.off_slab_tail);
  a.slab_dead = c->at<int32_t>(p.off_slab_dead);
  a.slab_inst = c->at<int32_t>(p.off_slab_inst);
  a.slab_k = c->at<int32_t>(p.off_slab_k);
  a.inst = c->at<DevInst>(p.off_inst);
  a.inj_cum = c->at<int64_t>(p.off_inj);
  a.e_edges = c->at<uint32_t>(p.off_edges);
  a.e_bucket = c->at<uint8_t>(p.off_edges + PIC_MAX_EBINS * 4);
  a.dens = c->at<uint64_t>(p.off_dens);
  a.cur = c->at<int64_t>(p.off_cur);
  a.counters = c->at<int64_t>(p.off_counters);
  a.queue = c->at<int32_t>(p.off_queue);
  a.status = c->at<uint32_t>(p.off_status);
  a.stats = c->at<unsigned long long>(p.off_stats);
  a.gen = c->at<uint64_t>(p.off_gen);
  a.etab = c->at<double>(p.off_etab);
  a.etab_words = p.etab_max;
  a.wt = c->at<uint32_t>(p.off_w);
  a.lds_etab_at = -1;
  a.lds_stage_at = -1;
  a.lds_stage1_at = -1;
  a.n_slabs = (int32_t)p.slab_inst.size();
  a.n_inst = c->cfg.n_instances;
  a.n_ebins = c->cfg.n_ebins;
  a.n_steps = c->cfg.n_steps;
  a.step = n;
  a.key0 = (uint32_t)c->cfg.seed;
  a.key1 = (uint32_t)(c->cfg.seed >> 32);
  a.e_min = c->cfg.e_min_fx;
  a.dt = c->cfg.dt;
  a.h = 0.5 * c->cfg.dt;
  a.tau_exp2 = c->cfg.tau_exp == 2;
  a.secondaries = (c->cfg.flags & PIC_F_SECONDARIES) != 0;
  a.absorb_next = (c->cfg.flags & PIC_F_ABSORB_NEXT) != 0;
  a.debug = p.debug;
  a.dens_on = (n % c->cfg.dens_stride) == 0;
  a.cur_on = (n % c->cfg.cur_stride) == 0;
  a.dens_slot = n / c->cfg.dens_stride;
  a.cur_slot = n / c->cfg.cur_stride;
  a.dens_lds = c->dens_lds;
  // the density histogram occupies LDS only on the steps that deposit density
  a.lds_dens_words = a.dens_on ? c->lds_dens_words : 0;
  a.lds_cur_words = c->lds_cur_words;
  a.inst_bytes = c->inst_bytes;
  a.z_phase = 0;
  a.z_write = 1;
  return a;
}

CompactArgs compact_args(const pic_ctx* c) {
  const Plan& p = c->plan;
  CompactArgs a;
  a.z = c->at<void>(p.off_z);
  a.mu = c->at<void>(p.off_mu);
  a.E = c->at<uint32_t>(p.off_E);
  a.uid = c->at<uint64_t>(p.off_uid);
  a.flags = c->at<uint32_t>(p.off_flags);
  a.ev = c->at<uint64_t>(p.off_ev);
  a.slab_base = c->at<int64_t>(p.off_slab_base);
  a.slab_tail = c->at<int32_t>(p.off_slab_tail);
  a.slab_dead = c->at<int32_t>(p.off_slab_dead);
  a.n_slabs = (int32_t)p.slab_inst.size();
  a.frac = c->tune.compact_frac;
  a.S = nullptr;
  a.K = 0;
  a.r = nullptr;
  a.w = c->at<uint32_t>(p.off_w);
  return a;
}

// Enqueue steps start .. start+n-1 of the forward run (adj_pass 0) or of a pass of the
// whole-tree adjoint replayed by the step kernel (adj_pass 1: tree returns, 2: scores;
// g_dens / g_cur the loss weights); same launch structure and tuning in every case.
pic_status enqueue_steps(pic_ctx* c, int start, int n, int adj_pass = 0,
                         const double* g_dens = nullptr, const double* g_cur = nullptr) {
  const bool fp64 = c->plan.state_bytes == 8;
  const int n_slabs = (int)c->plan.slab_inst.size();
  int grid = c->tune.grid > 0 ? c->tune.grid : 512;
  grid = std::max(1, std::min(grid, n_slabs));
  const int T = std::max(1, std::min(c->tune.sub_steps, kMaxSub));
  // write-back period: a multiple of the steps per launch; the adjoint passes, which move
  // more bytes per carrier than the forward, store z as rarely as the stamps allow
  int K = std::max(1, std::min(adj_pass ? kMaxZEvery : c->tune.z_every, kMaxZEvery));
  K = std::min(kMaxZEvery / T * T, (K + T - 1) / T * T);
  for (int s = start; s < start + n;) {
    // launches of T steps, aligned to the call's start; the write-back periods are
    // multiples of T, so only the last sub-step of a launch ever stores z
    int ns = std::min(T, start + n - s);
    StepArgs a = step_args(c, s);
    if (adj_pass) {
      a.adj_pass = adj_pass;
      a.adj_r = c->at<double>(c->plan.off_r);
      a.adj_R = c->at<double>(c->plan.off_R);
      a.adj_gd = g_dens;
      a.adj_gc = g_cur;
      a.adj_grad = c->at<double>(c->plan.off_grad);
      a.adj_K = c->plan.K;
      a.gen = nullptr;
    }
    int dens_on[kMaxSub] = {0, 0}, cur_on[kMaxSub] = {0, 0};
    for (int j = 0; j < kMaxSub; ++j) {
      const int sj = s + j;
      dens_on[j] = j < ns && (sj % c->cfg.dens_stride) == 0;
      cur_on[j] = j < ns && (sj % c->cfg.cur_stride) == 0;
    }
    // Density slices are held as 16-bit counters (unweighted runs without energy tables;
    // the counts stay exact) where two 32-bit slices would cost a workgroup per CU, or where
    // one 32-bit slice leaves no room for copies of queued carriers that a 16-bit one does.
    bool dens16 = false;
    if (adj_pass == 0 && ns > 1 && (dens_on[0] || dens_on[1]) && c->dens_lds &&
        c->plan.off_w < 0 && c->plan.etab_max == 0) {
      if (dens_on[0] && dens_on[1]) {
        dens16 = step_layout(c, c->tune.block, ns, dens_on, cur_on, nullptr) + step_static_lds() >
                 lds_per_wg(c->tune.block);
      } else {
        StepArgs l32 = a, l16 = a;
        step_layout(c, c->tune.block, ns, dens_on, cur_on, &l32, false);
        step_layout(c, c->tune.block, ns, dens_on, cur_on, &l16, true);
        const int copies32 = (l32.lds_stage_at >= 0) + (l32.lds_stage1_at >= 0);
        const int copies16 = (l16.lds_stage_at >= 0) + (l16.lds_stage1_at >= 0);
        dens16 = copies16 > copies32;
      }
    }
    // one step at a time where two density slices do not fit next to each other, or where
    // the first step would have to store z
    const bool first_writes = (s - start) % K == K - 1 || s == start + n - 1;
    if (ns > 1 && (first_writes ||
                   step_layout(c, c->tune.block, ns, dens_on, cur_on, nullptr, dens16,
                               adj_pass) > c->max_lds)) {
      ns = 1;
      dens_on[1] = cur_on[1] = 0;
      dens16 = false;
    }
    a.n_sub = ns;
    for (int j = 0; j < kMaxSub; ++j) {
      const int sj = s + j;
      a.sub_dens_on[j] = dens_on[j];
      a.sub_cur_on[j] = cur_on[j];
      a.sub_dens_slot[j] = sj / c->cfg.dens_stride;
      a.sub_cur_slot[j] = sj / c->cfg.cur_stride;
      a.sub_z_phase[j] = (sj - start) % K;
      a.sub_z_write[j] = j < ns && (a.sub_z_phase[j] == K - 1 || sj == start + n - 1) ? 1 : 0;
    }
    a.z_phase = a.sub_z_phase[0];
    a.z_write = a.sub_z_write[0];
    StepLaunch L;
    std::memset(&L, 0, sizeof(L));
    L.grid = grid;
    L.block = c->tune.block;
    L.lds = step_layout(c, c->tune.block, ns, dens_on, cur_on, &a, dens16, adj_pass);
    hipEvent_t* ev = nullptr;
    if (c->timing && adj_pass == 0) {
      c->tev.emplace_back();
      c->tstep.push_back(s);
      c->tnsub.push_back(ns);
      ev = c->tev.back().data();
      for (int k = 0; k < 3; ++k) ev[k] = nullptr;
      for (int k = 0; k < 3; ++k) HIP_TRY(hipEventCreate(&ev[k]));
      for (int k = 0; k < 2; ++k) L.ev[k] = ev[k];
    }
    HIP_TRY(launch_step(a, fp64, L, c->stream));
    bool compact = false;
    for (int j = 0; j < ns; ++j)
      compact = compact || (c->tune.compact_every > 0 && (s + j + 1) % c->tune.compact_every == 0);
    if (compact && !c->plan.debug && s + ns < c->cfg.n_steps) {
      CompactArgs ca = compact_args(c);
      if (adj_pass == 1) ca.r = c->at<double>(c->plan.off_r);  // partial returns move along
      HIP_TRY(launch_compact(ca, fp64, c->stream));
    }
    if (ev) HIP_TRY(hipEventRecord(ev[2], c->stream));
    s += ns;
  }
  return PIC_OK;
}

pic_status upload_tables(pic_ctx* c) {
  const Plan& p = c->plan;
  const pic_config& cfg = c->cfg;
  c->h_inst.assign(cfg.n_instances, DevInst{});
  c->h_etab.assign((size_t)p.etab_len, 0.0);
  int max_tab = 1;
  for (int i = 0; i < cfg.n_instances; ++i) {
    const pic_instance& I = c->inst[i];
    DevInst& D = c->h_inst[i];
    std::memset(&D, 0, sizeof(D));
    for (int l = 0; l < I.n_layers; ++l) {
      D.lay[l] = make_double4(I.z_bound[l], I.z_bound[l + 1], I.inv_tau_el[l], 0.5 * (1.0 + I.P0[l]));
      for (int s = 0; s < 2; ++s)
        D.chan[l][s] = make_double2(I.v[I.ch_of[l][s]], I.inv_tau0[I.ch_of[l][s]]);
    }
    // speed ratios of constant speeds (with energy tables the kernels divide v(E) values)
    for (int l = 0; l < I.n_layers; ++l)
      for (int s = 0; s < 2; ++s) {
        const double v = I.v[I.ch_of[l][s]];
        D.ratio[l][s][0] = l + 1 < I.n_layers && !I.e_nodes ? I.v[I.ch_of[l + 1][s]] / v : 1.0;
        D.ratio[l][s][1] = l > 0 && !I.e_nodes ? I.v[I.ch_of[l - 1][s]] / v : 1.0;
      }
    D.e_nodes = I.e_nodes;
    D.e_scale = I.e_nodes ? I.e_scale : 0.0;
    D.etab_off = p.etab_off[i];
    D.n_ch = (uint8_t)I.n_channels;
    for (int ch = 0; ch < I.n_channels; ++ch)
      for (int k = 0; k < I.e_nodes; ++k) {
        c->h_etab[p.etab_off[i] + (int64_t)ch * I.e_nodes + k] = I.v_node[ch][k];
        c->h_etab[p.etab_off[i] + (int64_t)(I.n_channels + ch) * I.e_nodes + k] = I.r_node[ch][k];
      }
    const bool wtd = (cfg.flags & PIC_F_WEIGHTS) != 0;
    D.w_nodes = wtd ? I.w_nodes : 0;
    D.w_scale = wtd ? I.w_scale : 0.0;
    for (int s = 0; s < 2 && wtd; ++s)
      for (int k = 0; k < I.w_nodes; ++k)
        c->h_etab[p.etab_off[i] + 2 * (int64_t)I.n_channels * I.e_nodes + s * I.w_nodes + k] =
            I.w_node[s][k];
    D.T_scale = I.T_scale;
    D.inv_dz = I.inv_dz;
    D.src_lo = I.src_z_lo;
    D.src_hi = I.src_z_hi;
    D.src_lambda = I.src_lambda;
    D.src_cd = I.src_cd;
    D.src_up = I.src_up_frac;
    for (int s = 0; s < 2; ++s) {
      D.e_lo[s] = I.src_e_lo[s];
      D.e_span[s] = I.src_e_span[s];
    }
    D.n_layers = I.n_layers;
    D.t_entries = I.t_entries;
    D.nz = I.nz;
    D.n_slabs = p.n_slabs_of[i];
    D.slab0 = p.slab0_of[i];
    D.root_offset = I.root_offset;
    D.dens_off = p.dens_off[i];
    D.cur_off = p.cur_off[i];
    D.gen_off = p.gen_off[i];
    for (int k = 0; k < I.n_layers - 1; ++k)
      for (int d = 0; d < 2; ++d)
        for (int s = 0; s < 2; ++s) D.tt[k][d][s] = (uint8_t)I.tt_of[k][d][s];
    for (int l = 0; l < I.n_layers; ++l)
      for (int s = 0; s < 2; ++s) D.chi[l][s] = (uint8_t)I.ch_of[l][s];
    for (int t = 0; t < I.n_ttables; ++t)
      for (int e = 0; e < I.t_entries; ++e) D.T[t * I.t_entries + e] = I.T[t][e];
    max_tab = std::max(max_tab, I.n_ttables * I.t_entries);
  }
  c->inst_bytes = (int)((kInstHead + max_tab * 8 + 15) & ~15);
  HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_inst), c->h_inst.data(),
                         sizeof(DevInst) * c->h_inst.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_slab_base), p.slab_base.data(), p.slab_base.size() * 8,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_slab_cap), p.slab_cap.data(), p.slab_cap.size() * 4,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_slab_inst), p.slab_inst.data(), p.slab_inst.size() * 4,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_slab_k), p.slab_k.data(), p.slab_k.size() * 4,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_edges), cfg.e_edges, PIC_MAX_EBINS * 4,
                         hipMemcpyHostToDevice, c->stream));
  // energy-bin bucket table: the bin of the lower end of each bucket of 2^22 units
  c->h_ebkt.assign(kEBuckets, 0);
  for (int b = 0, k = 0; b < kEBuckets; ++b) {
    const uint64_t lo = (uint64_t)b << kEBucketShift;
    while (k + 1 < cfg.n_ebins && cfg.e_edges[k + 1] <= lo) ++k;
    c->h_ebkt[b] = (uint8_t)k;
  }
  HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_edges + PIC_MAX_EBINS * 4), c->h_ebkt.data(),
                         kEBuckets, hipMemcpyHostToDevice, c->stream));
  if (p.etab_len > 0)
    HIP_TRY(hipMemcpyAsync(c->at<void>(p.off_etab), c->h_etab.data(), c->h_etab.size() * 8,
                           hipMemcpyHostToDevice, c->stream));
  // the copies read pageable host memory; finish them before the host buffers can change
  HIP_TRY(hipStreamSynchronize(c->stream));
  return PIC_OK;
}

pic_status clear_state(pic_ctx* c) {
  const Plan& p = c->plan;
  const int64_t NS = (int64_t)p.slab_inst.size();
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_slab_tail), NS, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_slab_dead), NS, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_dens), p.dens_len * 2, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_cur), p.cur_len * 2, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_counters), (int64_t)c->cfg.n_steps * kNC * 2, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_queue), (int64_t)c->cfg.n_steps * 2, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_status), 16, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_stats), (int64_t)c->cfg.n_steps * 4, 0, c->stream));
  if (p.off_gen >= 0) HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_gen), p.gen_len * 2, 0, c->stream));
  c->step = 0;
  return PIC_OK;
}

}  // namespace

extern "C" {

const char* pic_last_error(void) { return g_err.c_str(); }

pic_status pic_workspace_size(const pic_config* cfg, int64_t* bytes) {
  pic_status st = validate(cfg);
  if (st != PIC_OK) return st;
  if (!bytes) return fail(PIC_EINVAL, "null output");
  *bytes = make_plan(cfg).bytes;
  return PIC_OK;
}

}  // extern "C"

// Workspace of the allocation-free set-up: one array per device, held by the process from
// the library's load on that device until it ends.  Host code never uses the array's name
// as an address: each device's copy is resolved once with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[PIC_STATIC_WORKSPACE_BYTES];

namespace {

pic_status init_ctx(const pic_config* cfg, void* workspace, int64_t workspace_bytes, void* stream,
                    pic_ctx** out) {
  pic_status st = validate(cfg);
  if (st != PIC_OK) return st;
  if (!out) return fail(PIC_EINVAL, "null output");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(PIC_EINVAL, "workspace must be 256-byte aligned");
  Plan plan = make_plan(cfg);
  if (workspace_bytes < plan.bytes)
    return fail(PIC_ENOMEM, "workspace too small: need " + std::to_string(plan.bytes) + " bytes");
  pic_ctx* c = new pic_ctx();
  c->cfg = *cfg;
  c->inst.assign(cfg->inst, cfg->inst + cfg->n_instances);
  c->cfg.inst = c->inst.data();
  c->plan = std::move(plan);
  c->stream = (hipStream_t)stream;
  c->ws = (uint8_t*)workspace;
  c->tune.block = 256;
  c->tune.grid = 1024;
  c->tune.compact_every = 8;
  c->tune.compact_frac = 0.15f;
  c->tune.use_graph = 1;
  c->tune.z_every = 4;
  c->tune.sub_steps = 1;
  // LDS per workgroup: the density slice and the current slice of the largest instance,
  // plus one newborn queue per wave.  The density histogram goes to LDS when it fits
  // next to the queues of a 256-thread block; otherwise density uses global atomics.
  int nz_max = 1;
  for (const auto& I : c->inst) nz_max = std::max(nz_max, I.nz);
  c->lds_cur_words = nz_max * 2;
  const int dens_words = nz_max * cfg->n_ebins * 2;
  c->lds_dens_words = dens_words;
  c->dens_lds = true;
  c->max_lds = device_lds_limit();
  if (lds_for(c, 256) > c->max_lds) {
    c->dens_lds = false;
    c->lds_dens_words = 0;
  }
  const int none[kMaxSub] = {0, 0}, cur0[kMaxSub] = {1, 0};
  if (step_layout(c, 64, 1, none, cur0, nullptr) > c->max_lds) {
    delete c;
    return fail(PIC_EINVAL, "too many depth bins for the LDS current histogram");
  }
  st = upload_tables(c);
  if (st == PIC_OK) st = clear_state(c);
  if (st != PIC_OK) {
    delete c;
    return st;
  }
  *out = c;
  return PIC_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices];             // device address of `scratch`, per device
const pic_ctx* g_static_owner[kMaxDevices];  // the live context using it, per device

}  // namespace

extern "C" {

pic_status pic_init(const pic_config* cfg, void* workspace, int64_t workspace_bytes, void* stream,
                    pic_ctx** out) {
  return init_ctx(cfg, workspace, workspace_bytes, stream, out);
}

pic_status pic_init_static(const pic_config* cfg, void* stream, pic_ctx** out) {
  pic_status st = validate(cfg);
  if (st != PIC_OK) return st;
  if (!out) return fail(PIC_EINVAL, "null output");
  const int64_t need = make_plan(cfg).bytes;
  if (need > (int64_t)PIC_STATIC_WORKSPACE_BYTES)
    return fail(PIC_ENOMEM, "problem needs a workspace of " + std::to_string(need) +
                                " bytes, more than the static workspace of " +
                                std::to_string((int64_t)PIC_STATIC_WORKSPACE_BYTES) + " bytes");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PIC_EINVAL, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255)) return fail(PIC_EHIP, "static workspace address unusable");
    g_static_ptr[dev] = p;
  }
  if (g_static_owner[dev])
    return fail(PIC_ESTATE, "the static workspace of this device belongs to a live context "
                            "(pic_destroy it first)");
  pic_ctx* c = nullptr;
  st = init_ctx(cfg, g_static_ptr[dev], (int64_t)PIC_STATIC_WORKSPACE_BYTES, stream, &c);
  if (st != PIC_OK) return st;
  c->static_dev = dev;
  c->tune.use_graph = 0;  // instantiating a graph may allocate; steps launch directly
  g_static_owner[dev] = c;
  *out = c;
  return PIC_OK;
}

pic_status pic_inject(pic_ctx* c, const int64_t* sched) {
  if (!c || !sched) return fail(PIC_EINVAL, "null argument");
  const int NS = c->cfg.n_steps;
  std::vector<int64_t> cum((size_t)c->cfg.n_instances * (NS + 1));
  for (int i = 0; i < c->cfg.n_instances; ++i) {
    int64_t acc = 0;
    cum[(size_t)i * (NS + 1)] = 0;
    for (int n = 0; n < NS; ++n) {
      const int64_t v = sched[(size_t)i * NS + n];
      if (v < 0) return fail(PIC_EINVAL, "negative schedule entry");
      acc += v;
      cum[(size_t)i * (NS + 1) + n + 1] = acc;
    }
    if (acc != c->inst[i].n_primaries)
      return fail(PIC_EINVAL, "schedule of instance " + std::to_string(i) + " does not sum to n_primaries");
  }
  c->h_inj.swap(cum);
  HIP_TRY(hipMemcpyAsync(c->at<void>(c->plan.off_inj), c->h_inj.data(), c->h_inj.size() * 8,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->sched_set = true;
  return PIC_OK;
}

pic_status pic_step(pic_ctx* c, int32_t n) {
  if (!c) return fail(PIC_EINVAL, "null context");
  if (!c->sched_set) return fail(PIC_ESTATE, "pic_inject must precede pic_step");
  if (n < 0 || c->step + n > c->cfg.n_steps) return fail(PIC_EINVAL, "step count beyond n_steps");
  if (n == 0) return PIC_OK;
  const int start = c->step;
  if (c->tune.use_graph && n > 1 && !c->timing) {
    if (!(c->gexec && c->g_start == start && c->g_n == n)) {
      drop_graph(c);
      HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      pic_status st = enqueue_steps(c, start, n);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->stream, &g);
      if (st != PIC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      c->graph = g;
      HIP_TRY(hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
      c->g_start = start;
      c->g_n = n;
    }
    HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
  } else {
    pic_status st = enqueue_steps(c, start, n);
    if (st != PIC_OK) return st;
  }
  c->step += n;
  return PIC_OK;
}

pic_status pic_compact(pic_ctx* c) {
  if (!c) return fail(PIC_EINVAL, "null context");
  if (c->plan.debug) return PIC_OK;  // debug runs keep every record in place
  CompactArgs ca = compact_args(c);
  HIP_TRY(launch_compact(ca, c->plan.state_bytes == 8, c->stream));
  return PIC_OK;
}

pic_status pic_deposit(pic_ctx* c, double* dens_out, double* cur_out) {
  if (!c) return fail(PIC_EINVAL, "null context");
  HIP_TRY(launch_convert(c->at<uint64_t>(c->plan.off_dens), dens_out ? c->plan.dens_len : 0,
                         c->at<int64_t>(c->plan.off_cur), cur_out ? c->plan.cur_len : 0, dens_out,
                         cur_out, c->plan.off_w >= 0 ? 0x1p-16 : 1.0, c->stream));
  return PIC_OK;
}

pic_status pic_generations(pic_ctx* c, double* gen_out) {
  if (!c || !gen_out) return fail(PIC_EINVAL, "null argument");
  if (c->plan.off_gen < 0) return fail(PIC_ESTATE, "context created without PIC_F_GEN_MOMENT");
  HIP_TRY(launch_convert(c->at<uint64_t>(c->plan.off_gen), c->plan.gen_len, nullptr, 0, gen_out,
                         nullptr, c->plan.off_w >= 0 ? 0x1p-16 : 1.0, c->stream));
  return PIC_OK;
}

pic_status pic_counters(pic_ctx* c, int64_t* host_out) {
  if (!c) return fail(PIC_EINVAL, "null context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  uint32_t status = 0;
  HIP_TRY(hipMemcpy(&status, c->at<void>(c->plan.off_status), 4, hipMemcpyDeviceToHost));
  if (host_out)
    HIP_TRY(hipMemcpy(host_out, c->at<void>(c->plan.off_counters),
                      (size_t)c->cfg.n_steps * kNC * 8, hipMemcpyDeviceToHost));
  if (status & kStOverflow)
    return fail(PIC_ECAPACITY, "particle slots exhausted: raise capacity_factor");
  if (status & kStHits) return fail(PIC_ESTATE, "more than 8 boundary hits in one half step");
  return PIC_OK;
}

pic_status pic_reset(pic_ctx* c) {
  if (!c) return fail(PIC_EINVAL, "null context");
  return clear_state(c);
}

pic_status pic_set_tuning(pic_ctx* c, const pic_tuning* t) {
  if (!c || !t) return fail(PIC_EINVAL, "null argument");
  const int b = t->block;
  if (!(b == 64 || b == 128 || b == 256 || b == 512 || b == 1024))
    return fail(PIC_EINVAL, "block must be 64, 128, 256, 512 or 1024");
  if (t->grid < 0 || t->compact_every < 0 || !(t->compact_frac >= 0.0f && t->compact_frac <= 1.0f))
    return fail(PIC_EINVAL, "bad tuning");
  if (t->z_every < 1 || t->z_every > kMaxZEvery) return fail(PIC_EINVAL, "z_every must be 1..8");
  if (t->sub_steps < 1 || t->sub_steps > kMaxSub) return fail(PIC_EINVAL, "sub_steps must be 1 or 2");
  if (lds_for(c, b) > c->max_lds)
    return fail(PIC_EINVAL, "block too large for the LDS histograms of this configuration");
  c->tune = *t;
  drop_graph(c);
  return PIC_OK;
}

pic_status pic_get_tuning(const pic_ctx* c, pic_tuning* t) {
  if (!c || !t) return fail(PIC_EINVAL, "null argument");
  *t = c->tune;
  return PIC_OK;
}

pic_status pic_layout_of(const pic_ctx* c, pic_layout* o) {
  if (!c || !o) return fail(PIC_EINVAL, "null argument");
  const Plan& p = c->plan;
  o->n_slabs = (int64_t)p.slab_inst.size();
  o->capacity = p.capacity;
  o->off_z = p.off_z;
  o->off_mu = p.off_mu;
  o->off_E = p.off_E;
  o->off_uid = p.off_uid;
  o->off_flags = p.off_flags;
  o->off_ev = p.off_ev;
  o->off_slab_base = p.off_slab_base;
  o->off_slab_cap = p.off_slab_cap;
  o->off_slab_tail = p.off_slab_tail;
  o->off_slab_dead = p.off_slab_dead;
  o->off_slab_inst = p.off_slab_inst;
  o->off_dens = p.off_dens;
  o->off_cur = p.off_cur;
  o->off_counters = p.off_counters;
  o->dens_len = p.dens_len;
  o->cur_len = p.cur_len;
  o->state_bytes = p.state_bytes;
  o->flags_spin_shift = 0;
  o->flags_layer_shift = kLayerShift;
  o->flags_layer_bits = __builtin_popcount(kLayerMask);
  o->flags_gen_shift = kGenShift;
  o->flags_dead_bit = kDead;
  o->off_w = p.off_w;
  return PIC_OK;
}

// Clear the particle population only (the forward bins and counters stay).
static pic_status clear_particles(pic_ctx* c) {
  const Plan& p = c->plan;
  const int64_t NS = (int64_t)p.slab_inst.size();
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_slab_tail), NS, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_slab_dead), NS, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_queue), (int64_t)c->cfg.n_steps * 2, 0, c->stream));
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_status), 16, 0, c->stream));
  return PIC_OK;
}

// The whole-tree passes run in the step kernel's adjoint modes (two steps per launch, the
// forward's tuning) for runs without energy tables, weights or debug counts; the replay
// kernel k_adj covers the rest.
static bool tree_passes_in_step_kernel(const pic_ctx* c) {
  return c->plan.etab_max == 0 && c->plan.off_w < 0 && !c->plan.debug;
}

static pic_status replay(pic_ctx* c, int adj, const double* g_dens, const double* g_cur) {
  const Plan& p = c->plan;
  if (adj >= 2 && tree_passes_in_step_kernel(c)) {
    pic_status st = clear_particles(c);
    if (st != PIC_OK) return st;
    st = enqueue_steps(c, 0, c->cfg.n_steps, adj - 1, g_dens, g_cur);
    if (st != PIC_OK) return st;
    AdjArgs A;
    std::memset(&A, 0, sizeof(A));
    A.s = step_args(c, c->cfg.n_steps - 1);
    A.r = c->at<double>(p.off_r);
    A.R = c->at<double>(p.off_R);
    A.grad = c->at<double>(p.off_grad);
    A.K = p.K;
    A.n_ch = c->inst[0].n_channels;
    HIP_TRY(launch_adjoint_final(A, p.state_bytes == 8, adj, (uint32_t)c->cfg.n_steps, c->stream));
    return PIC_OK;
  }
  const bool fp64 = p.state_bytes == 8;
  const int n_slabs = (int)p.slab_inst.size();
  // at most 256 threads per workgroup; the grid keeps the forward's number of waves
  const int block = std::min(c->tune.block, 256);
  int grid = c->tune.grid > 0 ? c->tune.grid : 512;
  grid = (int)std::min<int64_t>((int64_t)grid * c->tune.block / block, 1 << 16);
  grid = std::max(1, std::min(grid, n_slabs));
  pic_status st = clear_particles(c);
  if (st != PIC_OK) return st;
  AdjArgs A;
  std::memset(&A, 0, sizeof(A));
  A.S = c->at<double>(p.off_S);
  A.r = c->at<double>(p.off_r);
  A.R = c->at<double>(p.off_R);
  A.g_dens = g_dens;
  A.g_cur = g_cur;
  A.grad = c->at<double>(p.off_grad);
  A.K = p.K;
  A.n_ch = c->inst[0].n_channels;
  CompactArgs ca = compact_args(c);
  ca.S = adj == 1 ? A.S : nullptr;
  ca.K = adj == 1 ? p.K : 0;
  ca.r = adj == 2 ? A.r : nullptr;
  // the replay advances one step per launch: z write-back at most every 4 steps and
  // compaction at least every 8 (longer periods pay in the forward's two-step launches
  // only), of slabs with at least 10 % dead slots (a compaction here also moves the
  // carriers' score rows or partial returns)
  ca.frac = std::max(ca.frac, 0.1f);
  const int K = std::max(1, std::min(c->tune.z_every, 4));
  const int compact_every =
      c->tune.compact_every > 0 ? std::min(c->tune.compact_every, 8) : 0;
  for (int n = 0; n < c->cfg.n_steps; ++n) {
    A.s = step_args(c, n);
    A.s.z_phase = n % K;
    A.s.z_write = (A.s.z_phase == K - 1 || n == c->cfg.n_steps - 1) ? 1 : 0;
    HIP_TRY(launch_adjoint(A, fp64, adj, grid, block, c->stream));
    // carriers move with their score rows (causal) or partial returns (tree pass 1)
    if (compact_every > 0 && (n + 1) % compact_every == 0 && n + 1 < c->cfg.n_steps)
      HIP_TRY(launch_compact(ca, fp64, c->stream));
  }
  A.s = step_args(c, c->cfg.n_steps - 1);
  HIP_TRY(launch_adjoint_final(A, fp64, adj, (uint32_t)c->cfg.n_steps, c->stream));
  return PIC_OK;
}

pic_status pic_backward(pic_ctx* c, const double* g_dens, const double* g_cur, double* grad_out,
                        int32_t estimator) {
  if (!c || !grad_out) return fail(PIC_EINVAL, "null argument");
  if (!c->sched_set) return fail(PIC_ESTATE, "pic_inject must precede pic_backward");
  const Plan& p = c->plan;
  if (estimator == 0 && p.off_S < 0)
    return fail(PIC_ESTATE, "causal adjoint needs a context created with adjoint 1 or 3");
  if (estimator == 1 && p.off_R < 0)
    return fail(PIC_ESTATE, "whole-tree adjoint needs a context created with adjoint 2 or 3");
  if (estimator != 0 && estimator != 1) return fail(PIC_EINVAL, "estimator must be 0 or 1");
  // the forward's graph stays: the replay enqueues its launches directly and changes
  // nothing that graph's launches were captured with, so a later forward reuses it
  HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_grad), (int64_t)p.K * 2, 0, c->stream));
  pic_status st;
  if (estimator == 0) {
    st = replay(c, 1, g_dens, g_cur);
  } else {
    HIP_TRY(launch_fill32(c->at<uint32_t>(p.off_R), std::max<int64_t>(p.n_roots, 1) * 2, 0, c->stream));
    st = replay(c, 2, g_dens, g_cur);
    if (st == PIC_OK) st = replay(c, 3, g_dens, g_cur);
  }
  if (st != PIC_OK) return st;
  HIP_TRY(hipMemcpyAsync(grad_out, c->at<void>(p.off_grad), (size_t)p.K * 8,
                         hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = c->cfg.n_steps;
  uint32_t status = 0;
  HIP_TRY(hipMemcpy(&status, c->at<void>(p.off_status), 4, hipMemcpyDeviceToHost));
  if (status & kStOverflow)
    return fail(PIC_ECAPACITY, "particle slots exhausted in the adjoint replay: raise capacity_factor");
  if (status & kStHits) return fail(PIC_ESTATE, "more than 8 boundary hits in one half step");
  return PIC_OK;
}

// Signature of a configuration for the tuning cache: every byte of the config struct and
// of the instance tables, plus the device.
static uint64_t config_signature(const pic_ctx* c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  pic_config cfg = c->cfg;
  cfg.inst = nullptr;
  mix(&cfg, sizeof(cfg));
  mix(c->inst.data(), c->inst.size() * sizeof(pic_instance));
  int dev = 0;
  (void)hipGetDevice(&dev);
  mix(&dev, sizeof(dev));
  return h;
}

static std::mutex g_tune_mu;
static std::map<uint64_t, pic_tuning> g_tune_cache;

// Time `steps` steps from a cleared state with the given tuning (ms on the stream).
static pic_status time_trial(pic_ctx* c, const pic_tuning& t, int steps, float* ms) {
  pic_status st = pic_set_tuning(c, &t);
  if (st != PIC_OK) return st;
  st = clear_state(c);
  if (st != PIC_OK) return st;
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  HIP_TRY(hipEventRecord(a, c->stream));
  st = enqueue_steps(c, 0, steps);
  HIP_TRY(hipEventRecord(b, c->stream));
  HIP_TRY(hipEventSynchronize(b));
  HIP_TRY(hipEventElapsedTime(ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

pic_status pic_autotune(pic_ctx* c, int32_t trial_steps, pic_tuning* best) {
  if (!c) return fail(PIC_EINVAL, "null context");
  if (!c->sched_set) return fail(PIC_ESTATE, "pic_inject must precede pic_autotune");
  const int steps = std::max(1, std::min<int>(trial_steps, c->cfg.n_steps));
  const uint64_t key = config_signature(c);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      pic_tuning t = it->second;
      if (c->static_dev >= 0) t.use_graph = 0;
      pic_status st = pic_set_tuning(c, &t);
      if (st != PIC_OK) return st;
      if (best) *best = t;
      return clear_state(c);
    }
  }
  pic_tuning cur = c->tune;
  cur.use_graph = 0;
  // the first stage times two-step launches (stage 3's usual choice), so that the
  // workgroup size suits the launches that will run: with one-step trials a 1024-thread
  // workgroup won on the batched workload, whose two-step launches it slows by 4 %
  cur.sub_steps = kMaxSub;
  cur.z_every = std::max(cur.z_every, kMaxSub);
  float best_ms = 1e30f;
  pic_tuning win = cur;
  // stage 1: workgroup size and persistent grid (a 1024-thread workgroup fills a CU alone:
  // one set of histogram slices per CU, so that LDS holds more queue copies beside them)
  for (int block : {128, 256, 512, 1024}) {
    if (lds_for(c, block) > c->max_lds) continue;
    for (int grid : {256, 512, 1024, 2048}) {
      pic_tuning t = cur;
      t.block = block;
      t.grid = grid;
      float ms = 0;
      pic_status st = time_trial(c, t, steps, &ms);
      if (st != PIC_OK) return st;
      if (ms < best_ms) {
        best_ms = ms;
        win = t;
      }
    }
  }
  // Stages 2 and 3 time longer prefixes: dead slots accumulate over the run, so the
  // compaction cadence and the write-back period show their effect only later.
  const int steps2 = std::min(c->cfg.n_steps, 4 * steps);
  {
    pic_status st = time_trial(c, win, steps2, &best_ms);
    if (st != PIC_OK) return st;
  }
  // stage 2: compaction cadence and threshold
  for (int every : {8, 16, 32, 64, 0}) {
    for (float frac : {0.05f, 0.1f, 0.25f}) {
      if (every == 0 && frac != 0.1f) continue;
      pic_tuning t = win;
      t.compact_every = every;
      t.compact_frac = frac;
      float ms = 0;
      pic_status st = time_trial(c, t, steps2, &ms);
      if (st != PIC_OK) return st;
      if (ms < best_ms) {
        best_ms = ms;
        win = t;
      }
    }
  }
  // stage 3: steps per launch and write-back period of z on the common path
  {
    const pic_tuning base = win;
    for (int ns : {1, 2}) {
      for (int k : {1, 2, 4, 8}) {
        if (k % ns) continue;
        pic_tuning t = base;
        t.sub_steps = ns;
        t.z_every = k;
        float ms = 0;
        pic_status st = time_trial(c, t, steps2, &ms);
        if (st != PIC_OK) return st;
        if (ms < best_ms) {
          best_ms = ms;
          win = t;
        }
      }
    }
  }
  // stage 4: the other of the two largest workgroup sizes with the settings chosen so far,
  // over the longer prefix (which of them wins depends on the histogram slices and queue
  // copies of the launches that stages 2 and 3 chose)
  if (win.block == 512 || win.block == 1024) {
    const pic_tuning base = win;
    const int other = base.block == 512 ? 1024 : 512;
    if (lds_for(c, other) <= c->max_lds) {
      for (int grid : {256, 512, 1024, 2048}) {
        pic_tuning t = base;
        t.block = other;
        t.grid = grid;
        float ms = 0;
        pic_status st = time_trial(c, t, steps2, &ms);
        if (st != PIC_OK) return st;
        if (ms < best_ms) {
          best_ms = ms;
          win = t;
        }
      }
    }
  }
  win.use_graph = 1;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = win;
  }
  if (c->static_dev >= 0) win.use_graph = 0;  // allocation-free contexts launch directly
  pic_status st = pic_set_tuning(c, &win);
  if (st != PIC_OK) return st;
  if (best) *best = win;
  return clear_state(c);
}

pic_status pic_time_kernels(pic_ctx* c, int32_t enable) {
  if (!c) return fail(PIC_EINVAL, "null context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  drop_events(c);
  c->timing = enable != 0;
  return PIC_OK;
}

pic_status pic_kernel_times(pic_ctx* c, double* out, int32_t max_steps, int32_t* n_out) {
  if (!c || !n_out || (max_steps > 0 && !out)) return fail(PIC_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (!out) {  // count only; the events stay
    *n_out = (int32_t)c->tev.size();
    return PIC_OK;
  }
  std::vector<unsigned long long> stats((size_t)c->cfg.n_steps * 2);
  HIP_TRY(hipMemcpy(stats.data(), c->at<void>(c->plan.off_stats), stats.size() * 8,
                    hipMemcpyDeviceToHost));
  const int n = std::min<int>((int)c->tev.size(), std::max(0, max_steps));
  for (int k = 0; k < n; ++k) {
    const auto& ev = c->tev[k];
    float f = 0, m = 0;
    HIP_TRY(hipEventElapsedTime(&f, ev[0], ev[1]));
    HIP_TRY(hipEventElapsedTime(&m, ev[1], ev[2]));
    const int s = c->tstep[k], ns = c->tnsub[k];
    double* o = out + (size_t)k * 6;
    o[0] = f;
    o[1] = m;
    o[2] = 0.0;
    o[3] = 0.0;
    for (int j = 0; j < ns; ++j) {
      o[2] += (double)stats[(size_t)(s + j) * 2];
      o[3] += (double)stats[(size_t)(s + j) * 2 + 1];
    }
    o[4] = s;
    o[5] = ns;
  }
  *n_out = (int32_t)c->tev.size();
  drop_events(c);
  return PIC_OK;
}

void pic_destroy(pic_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  drop_events(c);
  if (c->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
  }
  delete c;
}

}  // extern "C"
