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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
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


def alg_bytes(cnt: np.ndarray, fp64: bool) -> np.ndarray:
    """Algorithmic HBM bytes of each step launch, from the step counters.

    Per carrier alive at the start of the step: read z, cos(theta), E, uid, flags and
    write z.  Per event: write cos(theta) and E.  Per boundary hit: write cos(theta)
    (reflection) or the flags (transmission).  Per absorbed carrier: write its flags.
    Per appended carrier (new primary or secondary): write the whole state.
    """
    sz = 8 if fp64 else 4
    state = 2 * sz + 4 + 8 + 4
    alive_prev = np.concatenate([[0], cnt[:-1, 9]])
    ev = cnt[:, 1] + cnt[:, 2]
    hits = cnt[:, 6] + cnt[:, 7] + cnt[:, 8]
    appended = cnt[:, 0] + cnt[:, 3]
    return (alive_prev * (state + sz) + ev * (sz + 4) + hits * sz + cnt[:, 4] * 4
            + appended * state).astype(np.float64)


def particle_steps(cnt: np.ndarray) -> int:
    alive_prev = np.concatenate([[0], cnt[:-1, 9]])
    return int((alive_prev + cnt[:, 0]).sum())


def kernel_timing(sim, prob):
    """One extra run launched step by step with HIP events on the library's stream:
    mean duration of the step-kernel launch and algorithmic bytes per launch."""
    import torch

    tune = sim.tuning()
    every = tune["compact_every"]
    sim.set_tuning(use_graph=0, compact_every=0)
    sim.reset()
    st = sim.stream
    mk = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    s_ev = [mk() for _ in range(prob.n_steps)]
    e_ev = [mk() for _ in range(prob.n_steps)]
    comp = []
    for n in range(prob.n_steps):
        s_ev[n].record(st)
        sim.step(1)
        e_ev[n].record(st)
        if every and (n + 1) % every == 0 and n + 1 < prob.n_steps:
            a, b = mk(), mk()
            a.record(st)
            sim.compact()
            b.record(st)
            comp.append((a, b))
    st.synchronize()
    ms = np.array([s_ev[n].elapsed_time(e_ev[n]) for n in range(prob.n_steps)])
    comp_ms = float(sum(a.elapsed_time(b) for a, b in comp))
    cnt = sim.counters()
    sim.set_tuning(use_graph=tune["use_graph"], compact_every=every)
    return ms, cnt, comp_ms


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
                sample=f"first {roots} primaries of every instance ({n_roots} primary trees, "
                       f"{ps} particle-steps, {dt:.1f} s wall)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=["batched", "valve", "bilayer"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-roots", type=int, default=300)
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--tuning", default="", help="JSON dict of launch tuning")
    ap.add_argument("--slab", type=int, default=0)
    ap.add_argument("--tune-steps", type=int, default=60,
                    help="steps per autotuning trial (0: keep the default launch shape)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 4}))
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
        ms, cnt2, comp_ms = kernel_timing(sim, prob)
        assert np.array_equal(cnt2, cnt), "step-by-step run differs from the graph run"
        b = alg_bytes(cnt2, prob.state_fp64)
        achieved = b.sum() / (ms.sum() * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None)
        extra["step_kernel"] = dict(launches=int(prob.n_steps),
                                    mean_launch_ms=round(float(ms.mean()), 4),
                                    alg_bytes_per_launch=float(b.mean()),
                                    bytes_per_particle_step=round(float(b.sum() / ps), 2),
                                    compaction_ms_per_run=round(comp_ms, 3))
        print(f"[bench] step kernel: {ms.mean():.4f} ms/launch, {achieved:.1f} GB/s algorithmic",
              file=sys.stderr, flush=True)
    extra["tuning"] = sim.tuning()
    sim.close()

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
        "dtype": "f64",
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
