"""The standard workloads at their full sizes, in the benchmark's launch configuration
(autotuned shape, graph, compaction), checked against the oracle on a sample of primary
trees (trees are independent, so the oracle can follow any subset of them exactly) and
through identities that hold at any size: carrier-count conservation per step, density
sums equal to the live count, and exact energy conservation of the cascade."""
import sys

import numpy as np
import pytest

import workloads as W
from parity import compare_records

pytestmark = pytest.mark.gpu
C = dict(injected=0, ev_ee=1, ev_el=2, spawned=3, absorbed=4, sec_absorbed=5, transmit=6,
         refl_if=7, refl_surf=8, alive=9, e_absorbed=10)


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_full(prob, roots, oracle_mod, *, mono_energy=None):
    import torch
    from paper_1807_04733_amd import PicSim
    _say(f"[fullsize] {prob.name}: {prob.n_primaries} primaries, {len(prob.instances)} inst, "
         f"{prob.n_steps} steps")
    sim = PicSim(prob)
    sim.autotune(trial_steps=60)
    sim.step()
    cnt = sim.counters()
    dens, cur = sim.int_bins()
    parts = sim.particles(include_dead=False, roots_below=roots)
    e_alive = sim.alive_energy() if mono_energy is not None else None
    sim.close()
    torch.cuda.empty_cache()
    # identities at full size
    net = np.cumsum(cnt[:, C["injected"]] + cnt[:, C["spawned"]] - cnt[:, C["absorbed"]])
    assert np.array_equal(net, cnt[:, C["alive"]])
    assert cnt[:, C["injected"]].sum() == prob.n_primaries
    for n in range(0, prob.n_steps, prob.dens_stride):
        tot = sum(int(d[n // prob.dens_stride].sum()) for d in dens)
        assert tot == cnt[n, C["alive"]], n
    if mono_energy is not None:
        assert e_alive + int(cnt[:, C["e_absorbed"]].sum()) == mono_energy
    # sampled trees against the oracle
    ref = oracle_mod.run(prob, root_range=(0, roots), records=True)
    live = ref.records["dead"] < 0
    rr = {k: v[live] for k, v in ref.records.items()}
    r = compare_records(parts, rr, prob.state_fp64, z_tol=1e-9 if prob.state_fp64 else 0.0)
    _say(f"[fullsize] sample: joined {r['joined']} / dev {r['n_dev']} / ref {r['n_ref']}, "
         f"match {r['frac']:.6f}")
    assert r["joined"] >= 0.999 * r["n_ref"] and r["n_dev"] <= r["n_ref"] * 1.001 + 5
    assert r["frac"] >= 0.9999, r["bad"]
    return cnt


def test_bilayer_fp64_full(torch_gpu, oracle_mod):
    prob = W.config0()
    cnt = run_full(prob, 5000, oracle_mod, mono_energy=prob.n_primaries * W.e_fx(1.5))
    ref = oracle_mod.run(prob)
    assert np.array_equal(cnt, ref.counters)


@pytest.mark.parametrize("parallel", [True, False])
def test_spin_valve_full(torch_gpu, oracle_mod, parallel):
    run_full(W.config1(parallel=parallel), 2000, oracle_mod)


def test_batched_full(torch_gpu, oracle_mod):
    prob = W.config2()
    e0 = sum(int(it.n_primaries) * int(it.src_e_lo[0]) for it in prob.instances)
    run_full(prob, 60, oracle_mod, mono_energy=e0)


def test_adjoint_workload_forward_full(torch_gpu, oracle_mod):
    run_full(W.config3(), 1000, oracle_mod)


def test_multilayer_tables_full(torch_gpu, oracle_mod):
    run_full(W.config4(), 30, oracle_mod)


def test_multilayer_tables_adjoint_full(torch_gpu, oracle_mod):
    """Whole-tree adjoint of the full multilayer workload (2e8 primaries; 260 parameters:
    tau0 per channel and the nodes of the T(E) tables) with loss weights on the bins of the
    first 40 steps only.  Only the trees injected before step 40 then have a non-zero
    return, so the oracle, following exactly those trees over the whole run (their scores
    span all 2000 steps), must give the same gradient."""
    import torch
    from paper_1807_04733_amd import PicSim
    prob = W.config4()
    cut = 40
    rng = np.random.default_rng(11)
    gd, gc = [], []
    for i in range(len(prob.instances)):
        d = rng.normal(size=prob.dens_shape(i)) * (rng.uniform(size=prob.dens_shape(i)) < 0.2)
        d[(cut + prob.dens_stride - 1) // prob.dens_stride:] = 0.0
        c = rng.normal(size=prob.cur_shape(i)) * (rng.uniform(size=prob.cur_shape(i)) < 0.2)
        c[(cut + prob.cur_stride - 1) // prob.cur_stride:] = 0.0
        gd.append(d)
        gc.append(c)
    roots = int(prob.instances[0].sched[:cut].sum())
    assert all(int(it.sched[:cut].sum()) == roots for it in prob.instances)
    _say(f"[fullsize] {prob.name}: whole-tree adjoint, loss on steps < {cut} "
         f"({roots} trees per instance)")
    sim = PicSim(prob, adjoint=2)
    sim.step()
    sim.counters()
    g = sim.backward(gd, gc, 1)
    sim.close()
    torch.cuda.empty_cache()
    ref = oracle_mod.run(prob, root_range=(0, roots), g_dens=gd, g_cur=gc,
                         grad_per_tree=True).grad
    scale = np.abs(ref).max()
    _say(f"[fullsize] gradient: {int((ref != 0).sum())} non-zero of {ref.size}, "
         f"max |diff| / max |ref| = {np.abs(g - ref).max() / scale:.3e}")
    assert roots * len(prob.instances) > 10000 and scale > 0
    assert np.abs(g - ref).max() <= 1e-9 * scale
