"""Adjoint replay on the GPU vs the oracle's gradient on the same random streams (needs an
MI355X).  The comparison with common-random-number central differences at the stated size
is in test_gpu_adjoint_acceptance.py."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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


def _random_g(prob, seed, frac=0.05):
    rng = np.random.default_rng(seed)
    gd, gc = [], []
    for i in range(len(prob.instances)):
        d = rng.normal(size=prob.dens_shape(i)) * (rng.uniform(size=prob.dens_shape(i)) < frac)
        c = rng.normal(size=prob.cur_shape(i)) * (rng.uniform(size=prob.cur_shape(i)) < frac)
        gd.append(d)
        gc.append(c)
    return gd, gc


def _gpu_grad(prob, gd, gc, estimator, **kw):
    from paper_1807_04733_amd import PicSim
    it = prob.instances[0]
    K = it.n_channels + it.n_ttables * it.t_entries
    sim = PicSim(prob, adjoint=3 if K <= 16 else 2, **kw)
    sim.step()
    sim.counters()
    g = sim.backward(gd, gc, estimator)
    sim.close()
    return g


@pytest.mark.parametrize("estimator", [0, 1])
def test_gradient_matches_oracle_bilayer(torch_gpu, oracle_mod, estimator):
    prob = W.config3(n_primaries=6000, n_steps=90)
    gd, gc = _random_g(prob, 1)
    _say(f"[adjoint] config3-like, estimator {estimator}")
    g = _gpu_grad(prob, gd, gc, estimator, slab_primaries=1000, capacity_factor=30)
    ref = oracle_mod.run(prob, g_dens=gd, g_cur=gc, grad_per_tree=bool(estimator)).grad
    scale = np.abs(ref).max()
    _say(f"[adjoint] gpu {g}\n[adjoint] ref {ref}")
    assert scale > 0
    assert np.abs(g - ref).max() <= 1e-9 * scale


@pytest.mark.parametrize("estimator", [0, 1])
def test_gradient_with_compaction_every_step(torch_gpu, oracle_mod, estimator):
    """The forward and the replay compact after every step (the replay only slabs with at
    least 10 % tombstones), moving score rows (causal) or partial returns (whole-tree) with
    the carriers that fill the tombstones; the gradient still equals the oracle's."""
    prob = W.config3(n_primaries=5000, n_steps=90)
    prob.e_min_fx = W.e_fx(0.3)
    gd, gc = _random_g(prob, 5)
    g = _gpu_grad(prob, gd, gc, estimator, slab_primaries=500, capacity_factor=30,
                  tuning={"compact_every": 1, "compact_frac": 0.0})
    ref = oracle_mod.run(prob, g_dens=gd, g_cur=gc, grad_per_tree=bool(estimator)).grad
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(g - ref).max() <= 1e-9 * scale


@pytest.mark.parametrize("estimator", [0, 1])
def test_gradient_matches_oracle_removal_at_next_event(torch_gpu, oracle_mod, estimator):
    prob = W.config3(n_primaries=5000, n_steps=90)
    prob.e_min_fx = W.e_fx(0.3)
    prob.absorb_next = True
    gd, gc = _random_g(prob, 3)
    g = _gpu_grad(prob, gd, gc, estimator, slab_primaries=1000, capacity_factor=40)
    ref = oracle_mod.run(prob, g_dens=gd, g_cur=gc, grad_per_tree=bool(estimator)).grad
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(g - ref).max() <= 1e-9 * scale


@pytest.mark.parametrize("estimator", [0, 1])
def test_gradient_matches_oracle_energy_dependent_channels(torch_gpu, oracle_mod, estimator):
    """Speeds and inelastic rates from per-channel energy tables: the gradient with respect
    to ln tau0 (which scales the tabled rate) and the transmission nodes."""
    prob = W.variant(W.config3(n_primaries=5000, n_steps=90), energy_tables=True)
    gd, gc = _random_g(prob, 4)
    g = _gpu_grad(prob, gd, gc, estimator, slab_primaries=1000, capacity_factor=30)
    ref = oracle_mod.run(prob, g_dens=gd, g_cur=gc, grad_per_tree=bool(estimator)).grad
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(g - ref).max() <= 1e-9 * scale


@pytest.mark.parametrize("estimator", [0, 1])
def test_gradient_matches_oracle_weighted(torch_gpu, oracle_mod, estimator):
    """Weighted superparticles: every deposit term is scaled by the carrier's weight."""
    prob = W.variant(W.config3(n_primaries=5000, n_steps=90), weights=True)
    gd, gc = _random_g(prob, 5)
    g = _gpu_grad(prob, gd, gc, estimator, slab_primaries=1000, capacity_factor=30)
    ref = oracle_mod.run(prob, g_dens=gd, g_cur=gc, grad_per_tree=bool(estimator)).grad
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(g - ref).max() <= 1e-9 * scale


@pytest.mark.parametrize("block", [512, 1024])
def test_gradient_matches_oracle_batched_tables(torch_gpu, oracle_mod, block):
    """The whole-tree passes in the step kernel, in 512- and 1024-thread workgroups."""
    prob = W.config4(n_instances=2, primaries_per_instance=800, n_steps=300)
    gd, gc = _random_g(prob, 2, frac=0.02)
    g = _gpu_grad(prob, gd, gc, 1, slab_primaries=300, capacity_factor=30,
                  tuning={"block": block, "grid": 8, "sub_steps": 2, "z_every": 4})
    ref = oracle_mod.run(prob, g_dens=gd, g_cur=gc, grad_per_tree=True).grad
    scale = np.abs(ref).max()
    assert g.shape == ref.shape == (4 + 4 * 64,)
    assert np.abs(g - ref).max() <= 1e-9 * scale


@pytest.mark.parametrize("estimator", [0, 1])
def test_forward_after_backward_reuses_its_graph(torch_gpu, oracle_mod, estimator):
    """Forward (captured as a graph), adjoint replay, then the same forward again from a
    cleared state and a second replay: the second forward's counters and bins equal the
    first's and the oracle's, and both gradients equal the oracle's."""
    from paper_1807_04733_amd import PicSim
    prob = W.config3(n_primaries=3000, n_steps=60)
    gd, gc = _random_g(prob, 7)
    sim = PicSim(prob, adjoint=3, tuning={"block": 512, "grid": 64, "sub_steps": 2,
                                          "z_every": 4, "compact_every": 8, "use_graph": 1})
    runs = []
    for _ in range(2):
        sim.reset()
        sim.step()
        cnt = sim.counters()
        dens, cur = sim.int_bins()
        g = sim.backward(gd, gc, estimator)
        runs.append((cnt, dens[0], cur[0], g))
    sim.close()
    ref = oracle_mod.run(prob, g_dens=gd, g_cur=gc, grad_per_tree=estimator == 1)
    scale = np.abs(ref.grad).max()
    assert scale > 0
    for cnt, dens, cur, g in runs:
        assert np.array_equal(cnt, ref.counters)
        assert np.array_equal(dens, ref.dens[0])
        assert np.array_equal(cur, ref.cur[0])
        assert np.abs(g - ref.grad).max() <= 1e-9 * scale
