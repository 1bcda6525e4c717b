"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

`run(problem)` simulates a `workloads.Problem` with the oracle and returns the binned
density, spin current, per-step counters and, optionally, per-particle records and a
likelihood-ratio gradient.  `build()` compiles `pic_oracle.c` with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

COUNTER_NAMES = ("injected", "ev_ee", "ev_el", "spawned", "absorbed", "sec_absorbed", "transmit",
                 "refl_if", "refl_surf", "alive", "e_absorbed", "w_injected")
NCOUNTERS = len(COUNTER_NAMES)


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, OpenMP, no floating-point contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Instance(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32), ("n_channels", C.c_int32), ("n_ttables", C.c_int32),
        ("t_entries", C.c_int32),
        ("z_bound", C.POINTER(C.c_double)), ("ch_of", C.POINTER(C.c_int32)),
        ("v", C.POINTER(C.c_double)), ("inv_tau0", C.POINTER(C.c_double)),
        ("inv_tau_el", C.POINTER(C.c_double)), ("P0", C.POINTER(C.c_double)),
        ("T", C.POINTER(C.c_double)), ("tt_of", C.POINTER(C.c_int32)),
        ("T_scale", C.c_double),
        ("src_z_lo", C.c_double), ("src_z_hi", C.c_double), ("src_lambda", C.c_double),
        ("src_cd", C.c_double), ("src_up_frac", C.c_double),
        ("src_e_lo", C.c_uint32 * 2), ("src_e_span", C.c_uint32 * 2),
        ("sched", C.POINTER(C.c_int64)), ("root_offset", C.c_uint64),
        ("nz", C.c_int32), ("inv_dz", C.c_double),
        ("e_nodes", C.c_int32), ("e_scale", C.c_double),
        ("v_node", C.POINTER(C.c_double)), ("r_node", C.POINTER(C.c_double)),
        ("w_nodes", C.c_int32), ("w_scale", C.c_double), ("w_node", C.POINTER(C.c_double)),
    ]


class _Problem(C.Structure):
    _fields_ = [
        ("n_instances", C.c_int32), ("inst", C.POINTER(_Instance)), ("seed", C.c_uint64),
        ("dt", C.c_double), ("n_steps", C.c_int32), ("tau_exp", C.c_int32),
        ("e_min_fx", C.c_uint32), ("secondaries", C.c_int32), ("state_fp64", C.c_int32),
        ("n_ebins", C.c_int32), ("e_edges", C.POINTER(C.c_uint32)),
        ("dens_stride", C.c_int32), ("cur_stride", C.c_int32),
        ("root_lo", C.c_int64), ("root_hi", C.c_int64), ("n_threads", C.c_int32),
        ("absorb_next", C.c_int32), ("weighted", C.c_int32),
        ("script", C.POINTER(C.c_uint32)), ("n_script", C.c_int64),
    ]


class _Output(C.Structure):
    _fields_ = [
        ("dens", C.POINTER(C.c_uint64)), ("cur", C.POINTER(C.c_int64)),
        ("counters", C.POINTER(C.c_int64)),
        ("rec_cap", C.c_int64), ("n_rec", C.c_int64),
        ("rec_uid", C.POINTER(C.c_uint64)), ("rec_z", C.POINTER(C.c_double)),
        ("rec_mu", C.POINTER(C.c_double)), ("rec_E", C.POINTER(C.c_uint32)),
        ("rec_layer", C.POINTER(C.c_int32)), ("rec_spin", C.POINTER(C.c_int32)),
        ("rec_gen", C.POINTER(C.c_int32)), ("rec_dead", C.POINTER(C.c_int32)),
        ("rec_inst", C.POINTER(C.c_int32)), ("rec_ev", C.POINTER(C.c_int32)),
        ("rec_w", C.POINTER(C.c_uint32)),
        ("gen", C.POINTER(C.c_uint64)),
        ("g_dens", C.POINTER(C.c_double)), ("g_cur", C.POINTER(C.c_double)),
        ("grad", C.POINTER(C.c_double)), ("grad_per_tree", C.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = C.CDLL(LIB)
        _lib.orc_run.argtypes = [C.POINTER(_Problem), C.POINTER(_Output)]
        _lib.orc_run.restype = C.c_int
        _lib.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                           C.POINTER(C.c_uint32)]
        _lib.orc_philox4x32_10.restype = None
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one counter (4 words) under one key (2 words)."""
    lib = _load()
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib.orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


@dataclass
class OracleResult:
    dens: list          # per instance, shape problem.dens_shape(i), uint64 counts
    cur: list           # per instance, shape problem.cur_shape(i), int64 (2^-32 nm/fs)
    counters: np.ndarray  # (n_steps, NCOUNTERS) int64
    records: Optional[dict] = None
    grad: Optional[np.ndarray] = None
    gen: Optional[list] = None   # per instance, shape problem.gen_shape(i), uint64 sums

    def cur_float(self, i: int) -> np.ndarray:
        return self.cur[i].astype(np.float64) * 2.0 ** -32


def run(problem, *, records: bool = False, rec_cap: Optional[int] = None,
        root_range=None, n_threads: int = 0, g_dens=None, g_cur=None,
        grad_per_tree: bool = False, gen: Optional[bool] = None,
        script=None) -> OracleResult:
    """Simulate `problem` (a workloads.Problem) on the CPU.

    root_range=(lo, hi) restricts every instance to its local roots lo..hi-1 (trees are
    independent, so this is exactly the sub-population of a full run).  g_dens / g_cur
    (lists of arrays shaped like the bins) switch on the likelihood-ratio gradient of
    sum(g_dens*dens) + sum(g_cur*cur_float) with respect to (ln tau0 per channel, T table
    entries).  gen (default: problem.gen_moment) also returns the generation moment: the
    sum of the generation labels per (density slot, depth, spin).  script: rows of 8
    uint32 (a Philox counter, then the 4 words to return for it) that replace the
    generator's words for the listed counters (white-box tests).
    """
    lib = _load()
    if gen is None:
        gen = bool(getattr(problem, "gen_moment", False))
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a

    insts = (_Instance * len(problem.instances))()
    for i, it in enumerate(problem.instances):
        s = insts[i]
        s.n_layers = it.n_layers
        s.n_channels = it.n_channels
        s.n_ttables = it.n_ttables
        s.t_entries = it.t_entries
        s.z_bound = _ptr(arr(it.z_bound, np.float64), C.c_double)
        s.ch_of = _ptr(arr(it.ch_of, np.int32), C.c_int32)
        s.v = _ptr(arr(it.v, np.float64), C.c_double)
        s.inv_tau0 = _ptr(arr(it.inv_tau0, np.float64), C.c_double)
        s.inv_tau_el = _ptr(arr(it.inv_tau_el, np.float64), C.c_double)
        s.P0 = _ptr(arr(it.P0, np.float64), C.c_double)
        s.T = _ptr(arr(it.T, np.float64), C.c_double)
        s.tt_of = _ptr(arr(it.tt_of if it.tt_of.size else np.zeros(4, np.int32), np.int32),
                       C.c_int32)
        s.T_scale = it.T_scale
        s.src_z_lo, s.src_z_hi = it.src_z_lo, it.src_z_hi
        s.src_lambda, s.src_cd, s.src_up_frac = it.src_lambda, it.src_cd, it.src_up_frac
        s.src_e_lo[0], s.src_e_lo[1] = int(it.src_e_lo[0]), int(it.src_e_lo[1])
        s.src_e_span[0], s.src_e_span[1] = int(it.src_e_span[0]), int(it.src_e_span[1])
        s.sched = _ptr(arr(it.sched, np.int64), C.c_int64)
        s.root_offset = it.root_offset
        s.nz = it.nz
        s.inv_dz = it.inv_dz
        if getattr(it, "v_tab", None) is not None:
            s.e_nodes = int(it.v_tab.shape[1])
            s.e_scale = float(it.e_scale)
            s.v_node = _ptr(arr(it.v_tab, np.float64), C.c_double)
            s.r_node = _ptr(arr(it.r_tab, np.float64), C.c_double)
        if getattr(it, "w_tab", None) is not None:
            s.w_nodes = int(it.w_tab.shape[1])
            s.w_scale = float(it.w_scale)
            s.w_node = _ptr(arr(it.w_tab, np.float64), C.c_double)
    P = _Problem()
    P.n_instances = len(problem.instances)
    P.inst = insts
    P.seed = problem.seed
    P.dt = problem.dt
    P.n_steps = problem.n_steps
    P.tau_exp = problem.tau_exp
    P.e_min_fx = problem.e_min_fx
    P.secondaries = int(problem.secondaries)
    P.state_fp64 = int(problem.state_fp64)
    P.n_ebins = problem.n_ebins
    P.e_edges = _ptr(arr(problem.e_edges, np.uint32), C.c_uint32)
    P.dens_stride = problem.dens_stride
    P.cur_stride = problem.cur_stride
    P.root_lo, P.root_hi = (root_range if root_range is not None else (0, -1))
    P.n_threads = n_threads
    P.absorb_next = int(bool(getattr(problem, "absorb_next", False)))
    P.weighted = int(bool(getattr(problem, "weighted", False)))
    if script is not None:
        sc = arr(np.asarray(script, np.uint32).reshape(-1, 8), np.uint32)
        P.script = _ptr(sc, C.c_uint32)
        P.n_script = sc.shape[0]

    nd = [int(np.prod(problem.dens_shape(i))) for i in range(len(problem.instances))]
    nc = [int(np.prod(problem.cur_shape(i))) for i in range(len(problem.instances))]
    dens = np.zeros(sum(nd), np.uint64)
    cur = np.zeros(sum(nc), np.int64)
    counters = np.zeros((problem.n_steps, NCOUNTERS), np.int64)
    O = _Output()
    O.dens = _ptr(dens, C.c_uint64)
    O.cur = _ptr(cur, C.c_int64)
    O.counters = _ptr(counters, C.c_int64)
    ng = [int(np.prod(problem.gen_shape(i))) for i in range(len(problem.instances))]
    gen_arr = np.zeros(sum(ng), np.uint64) if gen else None
    if gen:
        O.gen = _ptr(gen_arr, C.c_uint64)
    rec = None
    if records:
        if rec_cap is None:
            n_roots = sum(it.n_primaries for it in problem.instances)
            if root_range is not None:
                n_roots = min(n_roots, (root_range[1] - root_range[0]) * len(problem.instances))
            rec_cap = max(1024, 64 * n_roots)
        rec = dict(uid=np.zeros(rec_cap, np.uint64), z=np.zeros(rec_cap),
                   mu=np.zeros(rec_cap), E=np.zeros(rec_cap, np.uint32),
                   layer=np.zeros(rec_cap, np.int32), spin=np.zeros(rec_cap, np.int32),
                   gen=np.zeros(rec_cap, np.int32), dead=np.zeros(rec_cap, np.int32),
                   inst=np.zeros(rec_cap, np.int32), ev=np.zeros((rec_cap, 4), np.int32),
                   w=np.zeros(rec_cap, np.uint32))
        O.rec_cap = rec_cap
        O.rec_uid = _ptr(rec["uid"], C.c_uint64)
        O.rec_z = _ptr(rec["z"], C.c_double)
        O.rec_mu = _ptr(rec["mu"], C.c_double)
        O.rec_E = _ptr(rec["E"], C.c_uint32)
        O.rec_layer = _ptr(rec["layer"], C.c_int32)
        O.rec_spin = _ptr(rec["spin"], C.c_int32)
        O.rec_gen = _ptr(rec["gen"], C.c_int32)
        O.rec_dead = _ptr(rec["dead"], C.c_int32)
        O.rec_inst = _ptr(rec["inst"], C.c_int32)
        O.rec_ev = _ptr(rec["ev"], C.c_int32)
        O.rec_w = _ptr(rec["w"], C.c_uint32)
    grad = None
    if g_dens is not None or g_cur is not None:
        inst0 = problem.instances[0]
        K = inst0.n_channels + inst0.n_ttables * inst0.t_entries
        grad = np.zeros(K)
        if g_dens is not None:
            gd = arr(np.concatenate([np.asarray(g, np.float64).ravel() for g in g_dens]),
                     np.float64)
            O.g_dens = _ptr(gd, C.c_double)
        if g_cur is not None:
            gc = arr(np.concatenate([np.asarray(g, np.float64).ravel() for g in g_cur]),
                     np.float64)
            O.g_cur = _ptr(gc, C.c_double)
        O.grad = _ptr(grad, C.c_double)
        O.grad_per_tree = int(grad_per_tree)
    rc = lib.orc_run(C.byref(P), C.byref(O))
    if rc != 0:
        raise RuntimeError(f"oracle failed with code {rc}")
    out_d, out_c = [], []
    od = oc = 0
    for i in range(len(problem.instances)):
        out_d.append(dens[od:od + nd[i]].reshape(problem.dens_shape(i)))
        out_c.append(cur[oc:oc + nc[i]].reshape(problem.cur_shape(i)))
        od += nd[i]
        oc += nc[i]
    out_g = None
    if gen:
        out_g, og = [], 0
        for i in range(len(problem.instances)):
            out_g.append(gen_arr[og:og + ng[i]].reshape(problem.gen_shape(i)))
            og += ng[i]
    if rec is not None:
        n = O.n_rec
        rec = {k: v[:n] for k, v in rec.items()}
    return OracleResult(out_d, out_c, counters, rec, grad, out_g)
