"""Python binding of libpic: argument marshalling around the C ABI.

Every step of the particle update runs in the HIP kernels of libpic.so; PyTorch only
provides the device workspace, the output tensors and the stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _abi


def make_config(problem, *, debug: bool = False, slab_primaries: int = 0,
                capacity_factor: float = 0.0, adjoint: int = 0):
    """Translate a workloads.Problem into the C structs (returns config and a keep-alive)."""
    insts = (_abi.PicInstance * len(problem.instances))()
    for i, it in enumerate(problem.instances):
        s = insts[i]
        L = it.n_layers
        if L > _abi.MAX_LAYERS or it.n_channels > _abi.MAX_CHANNELS:
            raise ValueError("instance exceeds the library's table limits")
        s.n_layers, s.n_channels = L, it.n_channels
        s.n_ttables, s.t_entries = it.n_ttables, it.t_entries
        for l in range(L + 1):
            s.z_bound[l] = float(it.z_bound[l])
        for l in range(L):
            s.ch_of[l][0], s.ch_of[l][1] = int(it.ch_of[l, 0]), int(it.ch_of[l, 1])
            s.inv_tau_el[l] = float(it.inv_tau_el[l])
            s.P0[l] = float(it.P0[l])
        for c in range(it.n_channels):
            s.v[c] = float(it.v[c])
            s.inv_tau0[c] = float(it.inv_tau0[c])
        for k in range(L - 1):
            for d in range(2):
                for sp in range(2):
                    s.tt_of[k][d][sp] = int(it.tt_of[k, d, sp])
        for t in range(it.n_ttables):
            for e in range(it.t_entries):
                s.T[t][e] = float(it.T[t, e])
        s.T_scale = float(it.T_scale)
        s.src_z_lo, s.src_z_hi = float(it.src_z_lo), float(it.src_z_hi)
        s.src_lambda, s.src_cd = float(it.src_lambda), float(it.src_cd)
        s.src_up_frac = float(it.src_up_frac)
        for sp in range(2):
            s.src_e_lo[sp] = int(it.src_e_lo[sp])
            s.src_e_span[sp] = int(it.src_e_span[sp])
        s.n_primaries = int(it.n_primaries)
        s.root_offset = int(it.root_offset)
        s.nz = int(it.nz)
        s.inv_dz = float(it.inv_dz)
        v_tab = getattr(it, "v_tab", None)
        if v_tab is not None:
            # energy-dependent channels: speed and relative inelastic rate per node
            n = int(v_tab.shape[1])
            s.e_nodes = n
            s.e_scale = float(it.e_scale)
            for c in range(it.n_channels):
                for k in range(n):
                    s.v_node[c][k] = float(v_tab[c, k])
                    s.r_node[c][k] = float(it.r_tab[c, k])
        w_tab = getattr(it, "w_tab", None)
        if w_tab is not None:
            # superparticle weights per (spin, node)
            s.w_nodes = int(w_tab.shape[1])
            s.w_scale = float(it.w_scale)
            for sp in range(2):
                for k in range(s.w_nodes):
                    s.w_node[sp][k] = float(w_tab[sp, k])
    cfg = _abi.PicConfig()
    cfg.n_instances = len(problem.instances)
    cfg.inst = insts
    cfg.seed = int(problem.seed)
    cfg.dt = float(problem.dt)
    cfg.n_steps = int(problem.n_steps)
    cfg.tau_exp = int(problem.tau_exp)
    cfg.e_min_fx = int(problem.e_min_fx)
    flags = 0
    if problem.state_fp64:
        flags |= _abi.F_STATE_FP64
    if problem.secondaries:
        flags |= _abi.F_SECONDARIES
    if debug:
        flags |= _abi.F_DEBUG
    if getattr(problem, "gen_moment", False):
        flags |= _abi.F_GEN_MOMENT
    if getattr(problem, "absorb_next", False):
        flags |= _abi.F_ABSORB_NEXT
    if getattr(problem, "weighted", False):
        flags |= _abi.F_WEIGHTS
    cfg.flags = flags
    if problem.n_ebins > _abi.MAX_EBINS:
        raise ValueError("too many energy bins")
    cfg.n_ebins = problem.n_ebins
    for k, e in enumerate(problem.e_edges):
        cfg.e_edges[k] = int(e)
    cfg.dens_stride = int(problem.dens_stride)
    cfg.cur_stride = int(problem.cur_stride)
    cfg.slab_primaries = int(slab_primaries)
    cfg.capacity_factor = float(capacity_factor)
    cfg.adjoint = int(adjoint)
    return cfg, insts


def workspace_bytes(problem, **kw) -> int:
    cfg, keep = make_config(problem, **kw)
    n = C.c_int64()
    _abi.check(_abi.load().pic_workspace_size(C.byref(cfg), C.byref(n)))
    return n.value


class PicSim:
    """One simulation context on a GPU (a thin owner of the workspace and the handle)."""

    def __init__(self, problem, *, device="cuda", debug: bool = False,
                 slab_primaries: int = 0, capacity_factor: float = 0.0, stream=None,
                 tuning: Optional[dict] = None, adjoint: int = 0,
                 static_workspace: bool = False):
        """static_workspace=True sets up with pic_init_static (the library's own device
        array, no allocation; one such context per device at a time); the inspection
        helpers that read the workspace (int_bins, particles, alive_energy) are then not
        available."""
        import torch

        self.problem = problem
        self.lib = _abi.load()
        self.device = torch.device(device)
        self._cfg, self._keep = make_config(problem, debug=debug,
                                            slab_primaries=slab_primaries,
                                            capacity_factor=capacity_factor, adjoint=adjoint)
        n = C.c_int64()
        _abi.check(self.lib.pic_workspace_size(C.byref(self._cfg), C.byref(n)))
        self.ws_bytes = n.value
        # a stream of our own (default priority): the legacy NULL stream cannot be
        # captured into a graph
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.handle = C.c_void_p()
        if static_workspace:
            self._raw = self.ws = None
            with torch.cuda.device(self.device):
                _abi.check(self.lib.pic_init_static(C.byref(self._cfg),
                                                    C.c_void_p(self.stream.cuda_stream),
                                                    C.byref(self.handle)))
        else:
            with torch.cuda.stream(self.stream):
                raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            shift = (-raw.data_ptr()) % 256
            if shift % 8:
                raise RuntimeError("workspace allocation is not 8-byte aligned")
            self._raw = raw
            self.ws = raw[shift:shift + self.ws_bytes]
            _abi.check(self.lib.pic_init(C.byref(self._cfg), C.c_void_p(self.ws.data_ptr()),
                                         C.c_int64(self.ws_bytes),
                                         C.c_void_p(self.stream.cuda_stream),
                                         C.byref(self.handle)))
        sched = np.ascontiguousarray(np.stack([it.sched for it in problem.instances]), np.int64)
        _abi.check(self.lib.pic_inject(self.handle, sched.ctypes.data_as(C.POINTER(C.c_int64))))
        self.layout = _abi.PicLayout()
        _abi.check(self.lib.pic_layout_of(self.handle, C.byref(self.layout)))
        if tuning:
            self.set_tuning(**tuning)

    # ---------------------------------------------------------------- driving
    def step(self, n: Optional[int] = None):
        if n is None:
            n = self.problem.n_steps
        _abi.check(self.lib.pic_step(self.handle, int(n)))

    def compact(self):
        _abi.check(self.lib.pic_compact(self.handle))

    def reset(self):
        _abi.check(self.lib.pic_reset(self.handle))

    def tuning(self) -> dict:
        t = _abi.PicTuning()
        _abi.check(self.lib.pic_get_tuning(self.handle, C.byref(t)))
        return {k: getattr(t, k) for k, _ in t._fields_}

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        t = _abi.PicTuning(**cur)
        _abi.check(self.lib.pic_set_tuning(self.handle, C.byref(t)))

    def autotune(self, trial_steps: int = 20) -> dict:
        t = _abi.PicTuning()
        _abi.check(self.lib.pic_autotune(self.handle, int(trial_steps), C.byref(t)))
        return {k: getattr(t, k) for k, _ in t._fields_}

    def time_kernels(self, enable: bool = True) -> None:
        """Record HIP events around each step launch and its compaction on the following
        steps (launched directly, no graph)."""
        _abi.check(self.lib.pic_time_kernels(self.handle, 1 if enable else 0))

    def kernel_times(self) -> np.ndarray:
        """Rows per timed launch: ms of the step launch, ms of the compaction after it,
        carrier-steps on the common path, carrier-steps on the general path, first step,
        number of steps."""
        n = C.c_int32(0)
        _abi.check(self.lib.pic_kernel_times(self.handle, None, 0, C.byref(n)))
        out = np.zeros((max(n.value, 1), 6), dtype=np.float64)
        _abi.check(self.lib.pic_kernel_times(
            self.handle, out.ctypes.data_as(C.POINTER(C.c_double)), n.value, C.byref(n)))
        return out[:n.value]

    @property
    def n_params(self) -> int:
        it = self.problem.instances[0]
        return it.n_channels + it.n_ttables * it.t_entries

    def backward(self, g_dens=None, g_cur=None, estimator: int = 0) -> np.ndarray:
        """Likelihood-ratio gradient of sum(g_dens*dens) + sum(g_cur*cur) with respect to
        (ln tau0 per channel, T table nodes).  g_* are per-instance arrays shaped like
        the bins (or one flat array / device tensor each), or None."""
        import torch

        def flat(g):
            if g is None:
                return None
            if isinstance(g, (list, tuple)):
                g = torch.cat([torch.as_tensor(x, dtype=torch.float64).reshape(-1).to(self.device)
                               for x in g])
            return torch.as_tensor(g, dtype=torch.float64, device=self.device).reshape(-1).contiguous()

        # the loss weights are produced on the caller's stream (autograd's); the replay runs
        # on the library's stream, which first waits for everything queued there
        caller = torch.cuda.current_stream(self.device)
        gd = flat(g_dens)
        gc = flat(g_cur)
        if gd is not None and gd.numel() != self.layout.dens_len:
            raise ValueError("g_dens does not match the density bins")
        if gc is not None and gc.numel() != self.layout.cur_len:
            raise ValueError("g_cur does not match the current bins")
        grad = torch.zeros(self.n_params, dtype=torch.float64, device=self.device)
        self.stream.wait_stream(caller)
        for t in (gd, gc, grad):
            if t is not None:
                t.record_stream(self.stream)
        # pic_backward synchronizes the library stream before it returns
        _abi.check(self.lib.pic_backward(
            self.handle, C.c_void_p(gd.data_ptr() if gd is not None else 0),
            C.c_void_p(gc.data_ptr() if gc is not None else 0),
            C.c_void_p(grad.data_ptr()), int(estimator)))
        return grad.cpu().numpy()

    def counters(self) -> np.ndarray:
        out = np.zeros((self.problem.n_steps, _abi.NCOUNTERS), np.int64)
        _abi.check(self.lib.pic_counters(self.handle, out.ctypes.data_as(C.POINTER(C.c_int64))))
        return out

    def deposit(self):
        """Binary64 bins per instance: (dens list, cur list) of device tensors."""
        import torch

        lay = self.layout
        # outputs belong to the caller's stream: the conversion on the library stream waits
        # for their allocation, and the caller's stream waits for the conversion
        caller = torch.cuda.current_stream(self.device)
        d = torch.empty(lay.dens_len, dtype=torch.float64, device=self.device)
        c = torch.empty(lay.cur_len, dtype=torch.float64, device=self.device)
        self.stream.wait_stream(caller)
        _abi.check(self.lib.pic_deposit(self.handle, C.c_void_p(d.data_ptr()),
                                        C.c_void_p(c.data_ptr())))
        d.record_stream(self.stream)
        c.record_stream(self.stream)
        caller.wait_stream(self.stream)
        dens, cur = [], []
        od = oc = 0
        for i in range(len(self.problem.instances)):
            sd = self.problem.dens_shape(i)
            sc = self.problem.cur_shape(i)
            nd, nc = int(np.prod(sd)), int(np.prod(sc))
            dens.append(d[od:od + nd].view(sd))
            cur.append(c[oc:oc + nc].view(sc))
            od += nd
            oc += nc
        return dens, cur

    def generations(self):
        """Generation moment per instance (device tensors shaped problem.gen_shape(i)): the
        sum of the generation labels of the carriers in each density cell (the problem
        must have gen_moment set)."""
        import torch

        shapes = [self.problem.gen_shape(i) for i in range(len(self.problem.instances))]
        n = sum(int(np.prod(sh)) for sh in shapes)
        caller = torch.cuda.current_stream(self.device)
        g = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        self.stream.wait_stream(caller)
        _abi.check(self.lib.pic_generations(self.handle, C.c_void_p(g.data_ptr())))
        g.record_stream(self.stream)
        caller.wait_stream(self.stream)
        out, o = [], 0
        for sh in shapes:
            m = int(np.prod(sh))
            out.append(g[o:o + m].view(sh))
            o += m
        return out

    def int_bins(self):
        """The raw integer bins (uint64 counts, int64 2^-32 nm/fs) as host arrays."""
        import torch

        self._need_ws()
        self.stream.synchronize()
        lay = self.layout
        d = self.ws[lay.off_dens:lay.off_dens + 8 * lay.dens_len].view(torch.int64)
        c = self.ws[lay.off_cur:lay.off_cur + 8 * lay.cur_len].view(torch.int64)
        d = d.cpu().numpy().view(np.uint64)
        c = c.cpu().numpy()
        dens, cur = [], []
        od = oc = 0
        for i in range(len(self.problem.instances)):
            sd, sc = self.problem.dens_shape(i), self.problem.cur_shape(i)
            nd, nc = int(np.prod(sd)), int(np.prod(sc))
            dens.append(d[od:od + nd].reshape(sd))
            cur.append(c[oc:oc + nc].reshape(sc))
            od += nd
            oc += nc
        return dens, cur

    def particles(self, include_dead: bool = True, roots_below: Optional[int] = None) -> dict:
        """Copy the particle state out of the workspace (for inspection and tests).

        roots_below=R keeps only the carriers of each instance's first R primary trees
        (selected on the device, so that full-size runs can be sampled)."""
        import torch

        self._need_ws()
        self.stream.synchronize()
        lay = self.layout
        ws = self.ws
        ns = lay.n_slabs

        def arr(off, n, dt):
            nb = n * torch.tensor([], dtype=dt).element_size()
            return ws[off:off + nb].view(dt)

        base = arr(lay.off_slab_base, ns, torch.int64).cpu().numpy()
        tail = arr(lay.off_slab_tail, ns, torch.int32).cpu().numpy()
        inst = arr(lay.off_slab_inst, ns, torch.int32).cpu().numpy()
        fdt = torch.float64 if lay.state_bytes == 8 else torch.float32
        cap = lay.capacity
        with torch.cuda.stream(self.stream):
            tb = torch.from_numpy(base).to(self.device)
            tt = torch.from_numpy(tail.astype(np.int64)).to(self.device)
            slab_of = torch.repeat_interleave(torch.arange(ns, device=self.device), tt)
            start = torch.cumsum(tt, 0) - tt
            ti = tb[slab_of] + (torch.arange(slab_of.numel(), device=self.device) - start[slab_of])
            if roots_below is not None:
                offs = torch.tensor([it.root_offset for it in self.problem.instances],
                                    dtype=torch.int64, device=self.device)
                uid = arr(lay.off_uid, cap, torch.int64)[ti]
                root = uid & 0xFFFFFFFF
                inst_t = torch.from_numpy(inst.astype(np.int64)).to(self.device)[slab_of]
                keep = (root - offs[inst_t]) < roots_below
                ti = ti[keep]
                slab_of = slab_of[keep]
        self.stream.synchronize()
        slab_of = slab_of.cpu().numpy()
        z = arr(lay.off_z, cap, fdt)[ti].double().cpu().numpy()
        mu = arr(lay.off_mu, cap, fdt)[ti].double().cpu().numpy()
        E = arr(lay.off_E, cap, torch.int32)[ti].cpu().numpy().view(np.uint32)
        uid = arr(lay.off_uid, cap, torch.int64)[ti].cpu().numpy().view(np.uint64)
        fl = arr(lay.off_flags, cap, torch.int32)[ti].cpu().numpy().view(np.uint32)
        out = dict(z=z, mu=mu, E=E, uid=uid,
                   spin=((fl >> np.uint32(lay.flags_spin_shift)) & np.uint32(1)).astype(np.int32),
                   layer=((fl >> np.uint32(lay.flags_layer_shift)) &
                          np.uint32((1 << lay.flags_layer_bits) - 1)).astype(np.int32),
                   gen=((fl >> np.uint32(lay.flags_gen_shift)) & np.uint32(0xFF)).astype(np.int32),
                   dead=((fl & np.uint32(lay.flags_dead_bit)) != 0),
                   inst=inst[slab_of].astype(np.int32))
        if lay.off_w >= 0:
            out["w"] = arr(lay.off_w, cap, torch.int32)[ti].cpu().numpy().view(np.uint32)
        if lay.off_ev >= 0:
            ev = arr(lay.off_ev, cap, torch.int64)[ti].cpu().numpy().view(np.uint64)
            out["ev"] = np.stack([(ev >> np.uint64(16 * k)) & np.uint64(0xFFFF)
                                  for k in range(4)], axis=1).astype(np.int32)
        if not include_dead:
            keep = ~out["dead"]
            out = {k: v[keep] for k, v in out.items()}
        return out

    def alive_energy(self) -> int:
        """Sum of the fixed-point energies of all live carriers (inspection helper)."""
        import torch

        self._need_ws()
        self.stream.synchronize()
        lay = self.layout
        with torch.cuda.stream(self.stream):
            E = self.ws[lay.off_E:lay.off_E + 4 * lay.capacity].view(torch.int32)
            fl = self.ws[lay.off_flags:lay.off_flags + 4 * lay.capacity].view(torch.int32)
            base = self.ws[lay.off_slab_base:lay.off_slab_base + 8 * lay.n_slabs].view(torch.int64)
            tail = self.ws[lay.off_slab_tail:lay.off_slab_tail + 4 * lay.n_slabs].view(torch.int32)
            tt = tail.to(torch.int64)
            slab_of = torch.repeat_interleave(torch.arange(lay.n_slabs, device=self.device), tt)
            start = torch.cumsum(tt, 0) - tt
            ti = base[slab_of] + (torch.arange(slab_of.numel(), device=self.device) - start[slab_of])
            live = fl[ti] >= 0                      # dead bit is the sign bit
            tot = (E[ti].to(torch.int64) & 0xFFFFFFFF)[live].sum()
        self.stream.synchronize()
        return int(tot.item())

    def _need_ws(self):
        if self.ws is None:
            raise RuntimeError("a context on the static workspace has no workspace tensor")

    def close(self):
        if self.handle:
            self.lib.pic_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
