"""Benchmark of the hot-electron particle-in-cell step on one MI355X.

One benchmark step = one complete run of the workload (clear the state, inject the
primaries, advance every carrier through all time steps with deposition), with the
problem tables already resident in HBM.  The headline workload is the batched forward
run: 256 Fe/Au/Fe stacks with randomised thicknesses (Fe 5-20 nm, Au 20-200 nm),
log-uniform primaries (1e4-1e6 per stack), pump energies (0.8-2.0 eV), P/AP alignment and
+-30 % lifetime / transmission scales, 500 steps of 1 fs, FP32 state, binary64 decisions.

Printed: one JSON line with the throughput in particle-steps/s (one particle-step = one
carrier advanced by one time step), the HBM roofline of the step kernel measured with
HIP events on the library's stream, and the CPU oracle timed on a bounded root sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Optional

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# VALU issue ceiling: 256 CUs x 4 SIMDs, each issuing one wave64 VALU instruction per 4
# cycles (16 lanes per cycle; binary64 add/mul/fma and the 32x32->64 integer products run
# at this full rate on gfx950), at 2.4 GHz: 6.144e11 wave instructions per second.
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
METRIC = "particle-steps/s (batched fwd, fwd+adjoint) & %HBM roofline at oracle tol"


def workload(name: str):
    if name == "batched":
        return W.config2(), "batched_256_fe_au_fe: 256 Fe(5-20)/Au(20-200)/Fe(5-20) stacks, " \
                            "log-uniform 1e4-1e6 primaries each, 500 x 1 fs, FP32 state"
    if name == "valve":
        return W.config1(parallel=True), "fe15_au100_fe15_P: 1e7 primaries U(0.5,2) eV, " \
                                         "1000 x 0.5 fs, FP32 state"
    if name == "bilayer":
        return W.config0(), "fe15_au100_bilayer: 1e5 primaries at 1.5 eV, 300 x 1 fs, FP64 state"
    raise SystemExit(f"unknown workload {name}")


def alg_bytes(cnt: np.ndarray, fp64: bool, launches=None, z_every: int = 1,
              sub_steps: int = 1) -> np.ndarray:
    """HBM bytes the step kernel itself must move per launch, from the step counters (its
    temporal blocking and lazy z write-back included; compare method_bytes).

    `launches`: rows (..., carrier-steps on the general path, first step, number of
    steps) of the timed launches; one launch per step when None.  Per launch: the state
    (z, cos(theta), E, uid, flags) of every carrier alive at its start is read once.  z is
    written by every carrier alive at the end of a launch that ends a z write-back period
    (or the run), and once per general-path carrier-step, which also writes the flags in
    launches that do not end a period.  Per event: cos(theta) and E.  Per boundary hit:
    cos(theta) (reflection) or the flags (transmission).  Per absorbed carrier: its flags.
    Per appended carrier (new primary or secondary): the whole state.  Not counted: the
    flags rewrite that resets a write-back stamp, and the general path re-reading the
    state of the carriers it takes (from L2 in the common case).
    """
    sz = 8 if fp64 else 4
    state = 2 * sz + 4 + 8 + 4
    n = len(cnt)
    if launches is None:
        launches = np.stack([np.zeros(n), np.zeros(n), np.zeros(n), cnt[:, 9],
                             np.arange(n), np.ones(n)], axis=1)
    t = max(1, int(sub_steps))
    k = max(1, min(int(z_every), 8))
    k = min(8 // t * t, (k + t - 1) // t * t)
    alive = cnt[:, 9].astype(np.float64)
    ev = (cnt[:, 1] + cnt[:, 2]).astype(np.float64)
    hits = (cnt[:, 6] + cnt[:, 7] + cnt[:, 8]).astype(np.float64)
    appended = (cnt[:, 0] + cnt[:, 3]).astype(np.float64)
    out = []
    for row in launches:
        s0, m = int(row[4]), int(row[5])
        last = s0 + m - 1
        gen = float(row[3])
        ap = alive[s0 - 1] if s0 > 0 else 0.0
        write = (last % k == k - 1) or last == n - 1
        sl = slice(s0, last + 1)
        b = (ap * state + (alive[last] if write else 0.0) * sz + gen * sz
             + (0.0 if write else gen * 4) + ev[sl].sum() * (sz + 4) + hits[sl].sum() * sz
             + cnt[sl, 4].sum() * 4 + appended[sl].sum() * state)
        out.append(b)
    return np.array(out, dtype=np.float64)


def method_bytes(cnt: np.ndarray, fp64: bool, launches) -> np.ndarray:
    """The method's algorithmic bytes per launch (the roofline's per-unit figure): what a
    pass per time step must move for each particle-step -- read the state (z, cos(theta),
    E, uid, flags: 24 B in FP32), write z -- plus cos(theta) and E per event, cos(theta)
    per reflection and a whole state per created carrier (primary or secondary); 29 B per
    particle-step at the batched workload's rates.  The two-step kernel moves less than
    this (alg_bytes, and the measured traffic), so its achieved rate is an effective one."""
    sz = 8 if fp64 else 4
    state = 2 * sz + 4 + 8 + 4
    alive_prev = np.concatenate([[0], cnt[:-1, 9]]).astype(np.float64)
    units = alive_prev + cnt[:, 0]
    per_step = (units * (state + sz) + (cnt[:, 1] + cnt[:, 2]) * (sz + 4.0)
                + (cnt[:, 7] + cnt[:, 8]) * float(sz) + (cnt[:, 0] + cnt[:, 3]) * float(state))
    out = []
    for row in launches:
        s0, m = int(row[4]), int(row[5])
        out.append(float(per_step[s0:s0 + m].sum()))
    return np.array(out, dtype=np.float64)


def particle_steps(cnt: np.ndarray) -> int:
    alive_prev = np.concatenate([[0], cnt[:-1, 9]])
    return int((alive_prev + cnt[:, 0]).sum())


def kernel_timing(sim):
    """One extra run launched step by step with HIP events that the library records on
    its stream around each step launch and its compaction.  Returns rows (ms step launch,
    ms compaction, carriers whose step took the common path, carriers that took the
    general path) and the run's counters."""
    sim.reset()
    sim.time_kernels(True)
    sim.step()
    cnt = sim.counters()
    rows = sim.kernel_times()
    sim.time_kernels(False)
    return rows, cnt


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, roots: int):
    import oracle

    oracle.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    res = oracle.run(prob, root_range=(0, roots), n_threads=threads)
    dt = time.perf_counter() - t0
    ps = particle_steps(res.counters)
    n_roots = sum(min(roots, it.n_primaries) for it in prob.instances)
    return dict(value=ps / dt, unit="particle-steps/s", cores=threads, kind="oracle",
                cpu=cpu_model(),
                sample=f"first {roots} primaries of every instance ({n_roots} primary trees, "
                       f"{ps} particle-steps, {dt:.1f} s wall)")


def adjoint_leg(n_primaries: int, tune_steps: int, slab: int = 8192):
    """Plain single-instance forward and its causal adjoint on the Fe(15)/Au(80) bilayer
    (E0 ~ U(0.5, 2) eV, 400 x 1 fs): loss = L2 distance of the spin current at z = 80 nm
    to a target curve; the adjoint returns 8 gradients (4 tau0, 4 T)."""
    import torch
    from paper_1807_04733_amd import PicSim

    prob = W.config3(n_primaries=n_primaries)
    # the replay keeps every carrier ever created (7.3 per primary on average at this
    # workload, at most 20 per tree): 10 slots per primary over slabs of thousands of
    # primaries
    sim = PicSim(prob, device="cuda:0", adjoint=1, slab_primaries=slab, capacity_factor=10)
    if tune_steps > 0:
        sim.autotune(trial_steps=tune_steps)
    sim.step()
    sim.counters()
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step()
    cnt = sim.counters()
    t_fwd = time.perf_counter() - t0
    d, c = sim.deposit()
    js = c[0][:, 80, 0] - c[0][:, 80, 1]
    target = 0.9 * js
    g_cur = torch.zeros_like(c[0])
    g_cur[:, 80, 0] = 2 * (js - target)
    g_cur[:, 80, 1] = -2 * (js - target)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad = sim.backward(None, g_cur, 0)
    t_bwd = time.perf_counter() - t0
    ps = particle_steps(cnt)
    tuning = sim.tuning()
    sim.close()
    del d, c, g_cur
    torch.cuda.empty_cache()
    return dict(workload=f"fe15_au80_bilayer: {n_primaries:.0e} primaries U(0.5,2) eV, 400 x 1 fs, "
                         "FP32 state, L2 loss on the spin current at z = 80 nm, 8 parameters",
                particle_steps=ps, forward_s=round(t_fwd, 4), adjoint_s=round(t_bwd, 4),
                adjoint_over_forward=round(t_bwd / t_fwd, 3),
                fwd_plus_adjoint_particle_steps_per_s=2 * ps / (t_fwd + t_bwd),
                estimator="causal score rows, lazy non-event flush",
                tuning=tuning, grad=[float(x) for x in grad])


def multilayer_adjoint_leg(n_instances: int, tune_steps: int, tuning: Optional[dict] = None):
    """[Fe(10)/Au(30)]x5 multilayers, a 50 fs Gaussian pump (3.125e6 primaries per stack),
    T(E) tables of 64 nodes, 2000 x 0.5 fs: the forward run and its whole-tree adjoint over
    260 parameters (ln tau0 of 4 channels, 4 tables x 64 nodes).  Loss: L2 distance of the
    spin current over every (t, z) to a target curve (0.9 times the run's own).  By default
    8 stacks, one GPU's share of the 64-stack workload sharded over 8 GPUs by stack.  A
    given `tuning` replaces the autotuner (a fixed launch shape for profiling)."""
    import torch
    from paper_1807_04733_amd import PicSim

    prob = W.config4(n_instances=n_instances)
    sim = PicSim(prob, device="cuda:0", adjoint=2, tuning=tuning)
    if tuning is None and tune_steps > 0:
        # the pump peaks at step 200: tune on a prefix that holds most of it
        sim.autotune(trial_steps=max(tune_steps, 250))
    sim.step()
    sim.counters()
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step()
    cnt = sim.counters()
    t_fwd = time.perf_counter() - t0
    d, c = sim.deposit()
    g_cur = []
    for ci in c:
        js = ci[:, :, 0] - ci[:, :, 1]
        g = torch.zeros_like(ci)
        g[:, :, 0] = 2 * (js - 0.9 * js)
        g[:, :, 1] = -2 * (js - 0.9 * js)
        g_cur.append(g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad = sim.backward(None, g_cur, 1)
    t_bwd = time.perf_counter() - t0
    ps = particle_steps(cnt)
    tuning = sim.tuning()
    sim.close()
    del d, c, g_cur
    torch.cuda.empty_cache()
    return dict(workload=f"{n_instances} x [Fe(10)/Au(30)]x5, {prob.n_primaries:.3g} primaries "
                         "(50 fs Gaussian pump), T(E) tables of 64 nodes, 2000 x 0.5 fs, FP32 "
                         "state, L2 loss on the spin current, 260 parameters",
                particle_steps=ps, forward_s=round(t_fwd, 4), adjoint_s=round(t_bwd, 4),
                adjoint_over_forward=round(t_bwd / t_fwd, 3),
                fwd_plus_adjoint_particle_steps_per_s=2 * ps / (t_fwd + t_bwd),
                estimator="whole-tree return, two replays", tuning=tuning,
                grad_norm=float(np.linalg.norm(grad)))


def sequential_leg(prob, batched_s: float, tuning: dict):
    """The same stacks run one after another, one context and one graph each, with the
    batched run's launch tuning (workgroup size, grid, steps per launch, write-back and
    compaction cadence), so that only the batching differs."""
    import torch
    from dataclasses import replace as dc_replace
    from paper_1807_04733_amd import PicSim

    total = 0.0
    ps = 0
    for inst in prob.instances:
        one = dc_replace(prob, instances=[inst])
        sim = PicSim(one, device="cuda:0", tuning=tuning)
        sim.step()
        sim.counters()
        sim.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step()
        cnt = sim.counters()
        total += time.perf_counter() - t0
        ps += particle_steps(cnt)
        sim.close()
    torch.cuda.empty_cache()
    return dict(instances=len(prob.instances), sequential_s=round(total, 4),
                batched_s=round(batched_s, 4), batched_speedup=round(total / batched_s, 3),
                particle_steps=ps, tuning="the batched run's")


def variants_leg(prob, tuning: dict):
    """The batched workload with the physics switches of the paper's comparisons, one timed
    run each (same launch tuning as the headline run)."""
    import torch
    from paper_1807_04733_amd import PicSim

    out = {}
    cases = {
        "generation_moment": dict(gen_moment=True),
        "removal_at_next_event": dict(absorb_next=True),
        "elastic_30fs": dict(tau_el=30.0),
        "transparent_interfaces": dict(transparent=True),
        "no_secondaries": dict(secondaries=False),
        "energy_dependent_channels": dict(energy_tables=True),
        "weighted_superparticles": dict(weights=True),
    }
    for name, kw in cases.items():
        sim = PicSim(W.variant(prob, **kw), device="cuda:0")
        sim.set_tuning(**{k: v for k, v in tuning.items() if k != "use_graph"})
        sim.step()
        sim.counters()
        sim.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step()
        cnt = sim.counters()
        dt = time.perf_counter() - t0
        sim.close()
        torch.cuda.empty_cache()
        ps = particle_steps(cnt)
        out[name] = dict(particle_steps=ps, seconds=round(dt, 4), rate=round(ps / dt, 0))
        print(f"[bench] variant {name}: {ps / dt:.4g} particle-steps/s", file=sys.stderr,
              flush=True)
    return out


def summarize_trace(path: str):
    """Per-kernel statistics of a rocprofv3 --kernel-trace CSV (ms)."""
    import csv
    import collections

    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(list)
    for r in rows:
        agg[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    tot = sum(sum(v) for v in agg.values())
    print(f"{'kernel':64s} {'calls':>6s} {'total_ms':>10s} {'mean_ms':>9s} {'share':>6s}")
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        print(f"{k[:64]:64s} {len(v):6d} {sum(v):10.3f} {sum(v) / len(v):9.4f} {sum(v) / tot:6.1%}")
    steps = [x for k, v in agg.items() if "k_step" in k for x in v]
    if steps:
        print(f"all step-kernel launches: {len(steps)}, mean {sum(steps) / len(steps):.4f} ms")
        last = sorted(((int(r["Start_Timestamp"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
                       for r in rows if "k_step" in r["Kernel_Name"]))
        return last
    return None


# the step kernel and the host code that plans its launches (LDS layout, queue copies,
# 16-bit density slices, steps per launch), which changes what a launch does
KERNEL_SOURCES = ("paper_1807_04733_amd/csrc/pic_kernels.hip",
                  "paper_1807_04733_amd/csrc/pic_device.h",
                  "paper_1807_04733_amd/csrc/pic_internal.h",
                  "paper_1807_04733_amd/csrc/pic_api.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_batched_256_hbm_traffic.md")
SQ_FILE = os.path.join(ROOT, "profiles", "k_step_batched_256_sq_counters.md")


def kernel_source_hash() -> str:
    """Hash of the step kernel's code and of its launch planning: the source files with //
    comments and blank lines removed, so that a comment edit does not disown a counter
    summary."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        for line in open(os.path.join(ROOT, f), encoding="utf-8"):
            code = re.sub(r"//.*", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _profile_line(path: str, tag: str):
    """The key=value pairs of the machine-readable `tag:` line of a committed profile
    summary, if it was taken on the current kernel source (otherwise None)."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith(tag + ":"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("kernel_source") != kernel_source_hash():
        return None
    return vals


def measured_traffic():
    """HBM bytes per step launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source (otherwise None)."""
    vals = _profile_line(TRAFFIC_FILE, "traffic")
    if vals is None:
        return None
    fetch = float(vals["fetch_kib"]) * float(vals["fetch_scale"]) * 1024
    write = float(vals["write_kib"]) * float(vals["write_scale"]) * 1024
    return fetch + write


def measured_valu():
    """VALU wave instructions per step launch (SQ_INSTS_VALU) from the committed counter
    summary, if it was taken on the current kernel source (otherwise None)."""
    vals = _profile_line(SQ_FILE, "valu")
    return None if vals is None else float(vals["insts_per_launch"])


def summarize_pmc(path: str, last: int):
    """Mean of each counter per step-kernel dispatch over the last `last` dispatches of a
    rocprofv3 --pmc CSV (and the same for every other kernel)."""
    import csv
    import collections

    per = collections.defaultdict(lambda: collections.defaultdict(float))
    name = {}
    for r in csv.DictReader(open(path)):
        d = int(r["Dispatch_Id"])
        per[d][r["Counter_Name"]] += float(r["Counter_Value"])
        name[d] = r["Kernel_Name"]
    steps = sorted(d for d in per if "k_step" in name[d])
    sel = steps[-last:] if last else steps
    counters = sorted({c for d in (sel or per) for c in per[d]})
    print(f"step-kernel dispatches averaged: {len(sel)} (of {len(steps)})")
    for c in counters if sel else []:
        print(f"  {c}: {sum(per[d][c] for d in sel) / len(sel):.6g} per dispatch")
    # with several step-kernel instantiations (the forward and the adjoint passes): each
    # one over its own last `last` dispatches
    names = sorted({name[d] for d in steps})
    for k in names if len(names) > 1 else []:
        ds = [d for d in steps if name[d] == k]
        ds = ds[-last:] if last else ds
        for c in counters:
            vals = [per[d][c] for d in ds if c in per[d]]
            if vals:
                print(f"  [{k[:48]}] {c}: {sum(vals) / len(vals):.6g} per dispatch "
                      f"(last {len(vals)} of {sum(1 for d in steps if name[d] == k)})")
    for k in sorted(set(name.values())):
        if "k_step" in k:
            continue
        ds = [d for d in per if name[d] == k]
        for c in counters:
            vals = [per[d][c] for d in ds if c in per[d]]
            if vals:
                print(f"  [{k[:48]}] {c}: {sum(vals) / len(vals):.6g} per dispatch ({len(vals)})")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=["batched", "valve", "bilayer"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-roots", type=int, default=3000)
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--tuning", default="", help="JSON dict of launch tuning")
    ap.add_argument("--slab", type=int, default=0)
    ap.add_argument("--adjoint-slab", type=int, default=8192,
                    help="primaries per slab of the forward+adjoint leg (0: the default)")
    ap.add_argument("--tune-steps", type=int, default=60,
                    help="steps per autotuning trial (0: keep the default launch shape)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--adjoint-primaries", type=int, default=100_000_000,
                    help="primaries of the forward+adjoint leg (0: skip)")
    ap.add_argument("--multilayer-instances", type=int, default=8,
                    help="stacks of the multilayer forward + whole-tree adjoint leg (0: skip; "
                         "64: the whole workload)")
    ap.add_argument("--multilayer-only", action="store_true",
                    help="run only the multilayer forward + adjoint leg and print it")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip running the batched stacks one by one")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the physics-variant runs of the batched workload")
    ap.add_argument("--summarize-pmc", default="",
                    help="print per-dispatch counter means of a rocprofv3 --pmc CSV and exit")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the step kernel's sources and exit")
    ap.add_argument("--summarize-trace", default="",
                    help="print per-kernel statistics of a rocprofv3 kernel-trace CSV and exit")
    ap.add_argument("--last-launches", type=int, default=0,
                    help="with --summarize-trace: also report the mean of the last N step launches")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.last_launches)
        return
    if args.summarize_trace:
        last = summarize_trace(args.summarize_trace)
        if last and args.last_launches:
            tail = [d for _, d in last[-args.last_launches:]]
            print(f"last {len(tail)} step-kernel launches (the HIP-event timing run): "
                  f"mean {sum(tail) / len(tail):.4f} ms")
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4}))
        return
    if args.multilayer_only:
        print(json.dumps(multilayer_adjoint_leg(args.multilayer_instances, args.tune_steps,
                                                json.loads(args.tuning) if args.tuning else None)))
        return
    if args.gpus != 1:
        print("this build runs on one GPU only: the particle update is sharded across GPUs "
              "by instance / primary range with one all-reduce of the integer bins, which is "
              "not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1807_04733_amd import PicSim

    prob, desc = workload(args.workload)
    print(f"[bench] {desc}: building context", file=sys.stderr, flush=True)
    sim = PicSim(prob, device="cuda:0", slab_primaries=args.slab)
    if args.tuning:
        sim.set_tuning(**json.loads(args.tuning))
    elif args.tune_steps > 0:
        t0 = time.perf_counter()
        tuned = sim.autotune(trial_steps=args.tune_steps)
        print(f"[bench] autotuned in {time.perf_counter() - t0:.1f} s: {tuned}",
              file=sys.stderr, flush=True)
    for w in range(args.warmup):
        sim.reset()
        sim.step()
        cnt = sim.counters()
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    sim.stream.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    for k in range(args.steps):
        sim.reset()
        sim.step()
    stop.record(sim.stream)
    stop.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt = sim.counters()
    gpu_ms = start.elapsed_time(stop)
    ps = particle_steps(cnt)
    value = ps * args.steps / wall
    print(f"[bench] timed {args.steps} runs: {wall:.3f} s wall, {gpu_ms:.1f} ms on the stream, "
          f"{ps} particle-steps per run", file=sys.stderr, flush=True)

    roof = None
    extra = {}
    if not args.no_kernel_timing:
        rows, cnt2 = kernel_timing(sim)
        assert np.array_equal(cnt2, cnt), "step-by-step run differs from the graph run"
        tune = sim.tuning()
        b = alg_bytes(cnt2, prob.state_fp64, launches=rows, z_every=tune["z_every"],
                      sub_steps=tune["sub_steps"])
        mb = method_bytes(cnt2, prob.state_fp64, rows)
        ms, c_ms = rows[:, 0], rows[:, 1]
        achieved = mb.sum() / (ms.sum() * 1e-3) / 1e9
        moved = b.sum() / (ms.sum() * 1e-3) / 1e9
        traffic = measured_traffic() if args.workload == "batched" else None
        valu = measured_valu() if args.workload == "batched" else None
        launch_s = float(ms.mean()) * 1e-3
        # Two roofs for the step kernel.  HBM: the method's bytes per particle-step (the
        # algorithmic bytes) over the launch time -- an effective rate, since the two-step
        # kernel moves fewer bytes -- and beside it the measured traffic (rocprofv3
        # FETCH_SIZE + WRITE_SIZE per launch) as a fraction of the peak.  VALU: the wave
        # instructions per launch (SQ_INSTS_VALU) at the issue ceiling.  `bound` is the
        # nearer roof by measurement (measured traffic vs VALU), and the top-level
        # achieved / peak / frac are that roof's.
        hbm = dict(achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=round(achieved / HBM_PEAK_GBS, 4),
                   basis="method bytes per particle-step / launch time (effective)",
                   traffic_gbs=None, traffic_frac=None)
        if traffic is not None:
            tg = traffic / launch_s / 1e9
            hbm["traffic_gbs"] = round(tg, 1)
            hbm["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)
        valu_roof = None
        if valu is not None:
            vg = valu / launch_s / 1e9
            valu_roof = dict(achieved=round(vg, 1), peak=VALU_PEAK_GINST,
                             unit="G wave64 VALU instructions/s",
                             frac=round(vg / VALU_PEAK_GINST, 4), insts_per_launch=valu,
                             issue="1 wave64 instruction per SIMD per 4 cycles, "
                                   "1024 SIMDs, 2.4 GHz")
        roof = dict(bound="hbm", achieved=hbm["achieved"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=hbm["frac"], traffic=None if traffic is None else round(traffic, 0),
                    hbm=hbm, valu=valu_roof)
        if valu_roof is not None and hbm["traffic_frac"] is not None and \
                valu_roof["frac"] > hbm["traffic_frac"]:
            roof.update(bound="alu", achieved=valu_roof["achieved"], peak=VALU_PEAK_GINST,
                        unit=valu_roof["unit"], frac=valu_roof["frac"])
        left = float(rows[:, 3].sum() / max(1.0, rows[:, 2:4].sum()))
        extra["step_kernel"] = dict(kernel="k_step", launches=int(len(rows)),
                                    steps_per_launch=int(tune["sub_steps"]),
                                    mean_launch_ms=round(float(ms.mean()), 4),
                                    method_bytes_per_launch=float(mb.mean()),
                                    method_bytes_per_particle_step=round(float(mb.sum() / ps), 2),
                                    moved_bytes_per_launch=float(b.mean()),
                                    moved_bytes_per_particle_step=round(float(b.sum() / ps), 2),
                                    moved_gbs=round(moved, 1),
                                    general_path_fraction=round(left, 5),
                                    kernel_source=kernel_source_hash(),
                                    compaction_ms_per_run=round(float(c_ms.sum()), 3))
        print(f"[bench] step kernel: {ms.mean():.4f} ms/launch, {achieved:.1f} GB/s of the "
              f"method's bytes ({moved:.1f} GB/s of the kernel's own), general-path fraction "
              f"{left:.4f}", file=sys.stderr, flush=True)
    extra["tuning"] = sim.tuning()
    sim.close()
    torch.cuda.empty_cache()
    if args.workload == "batched" and not args.no_sequential:
        print("[bench] running the stacks one by one", file=sys.stderr, flush=True)
        extra["sequential"] = sequential_leg(prob, wall / args.steps,
                                             {k: v for k, v in extra["tuning"].items()})
        print(f"[bench] sequential: {extra['sequential']}", file=sys.stderr, flush=True)
    if args.workload == "batched" and not args.no_variants:
        print("[bench] physics variants", file=sys.stderr, flush=True)
        extra["variants"] = variants_leg(prob, extra["tuning"])
    if args.adjoint_primaries > 0:
        print("[bench] forward + adjoint leg", file=sys.stderr, flush=True)
        try:
            extra["adjoint"] = adjoint_leg(args.adjoint_primaries, args.tune_steps,
                                           args.adjoint_slab)
        except Exception as e:  # reported, never hidden
            extra["adjoint"] = {"error": str(e)}
        print(f"[bench] adjoint: {extra['adjoint']}", file=sys.stderr, flush=True)

    if args.multilayer_instances > 0:
        print("[bench] multilayer forward + whole-tree adjoint leg", file=sys.stderr, flush=True)
        try:
            extra["multilayer_adjoint"] = multilayer_adjoint_leg(args.multilayer_instances,
                                                                 args.tune_steps)
        except Exception as e:  # reported, never hidden
            extra["multilayer_adjoint"] = {"error": str(e)}
        print(f"[bench] multilayer adjoint: {extra['multilayer_adjoint']}", file=sys.stderr,
              flush=True)

    cpu = None
    if not args.no_cpu:
        print("[bench] timing the CPU oracle on a root sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(prob, args.cpu_roots)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 decisions, f32 state" if not prob.state_fp64 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "instances": len(prob.instances),
                   "primaries": prob.n_primaries, "time_steps": prob.n_steps,
                   "particle_steps_per_run": ps, "state": "fp64" if prob.state_fp64 else "fp32"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
