"""Device path vs the CPU oracle, through the C ABI (needs an MI355X).

Acceptance: per-particle final state and event counts (joined on uid) identical for
>= 99.99 % of particles; the integer bins identical, and the binary64 bins within
1e-5 relative L1.  Sizes span several slabs, several waves per slab and ragged tails.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from parity import compare_records, rel_l1

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


def run_both(prob, oracle_mod, *, debug=True, tuning=None, slab_primaries=0, records=True):
    from paper_1807_04733_amd import PicSim
    _say(f"[parity] {prob.name or 'problem'}: {prob.n_primaries} primaries, "
         f"{len(prob.instances)} inst, {prob.n_steps} steps, debug={debug}, tuning={tuning}")
    sim = PicSim(prob, debug=debug, slab_primaries=slab_primaries, tuning=tuning)
    sim.step()
    cnt = sim.counters()
    dens, cur = sim.int_bins()
    fd, fc = sim.deposit()
    fd = [x.cpu().numpy() for x in fd]
    fc = [x.cpu().numpy() for x in fc]
    parts = sim.particles() if records else None
    gen = [x.cpu().numpy() for x in sim.generations()] if prob.gen_moment else None
    sim.close()
    ref = oracle_mod.run(prob, records=records)
    return dict(cnt=cnt, dens=dens, cur=cur, fd=fd, fc=fc, parts=parts, gen=gen), ref


def assert_parity(dev, ref, prob, *, exact_bins=True):
    fp64 = prob.state_fp64
    if dev["parts"] is not None:
        r = compare_records(dev["parts"], ref.records, fp64, z_tol=1e-9 if fp64 else 0.0)
        _say(f"[parity] joined {r['joined']} / dev {r['n_dev']} / ref {r['n_ref']}, "
             f"match {r['frac']:.6f}")
        assert r["joined"] >= 0.999 * r["n_ref"]
        assert r["frac"] >= 0.9999, r["bad"]
    # weighted runs: integer density / generation bins in 2^-16 units of weight
    ds = 2.0 ** -16 if prob.weighted else 1.0
    if dev["parts"] is not None and prob.weighted:
        assert "w" in dev["parts"]
    for i in range(len(prob.instances)):
        assert rel_l1(dev["fd"][i], ref.dens[i] * ds) <= 1e-5
        assert rel_l1(dev["fc"][i], ref.cur_float(i)) <= 1e-5
        if exact_bins:
            assert np.array_equal(dev["dens"][i], ref.dens[i])
            assert np.array_equal(dev["cur"][i], ref.cur[i])
        if dev["gen"] is not None:
            assert np.array_equal(dev["gen"][i], ref.gen[i].astype(np.float64) * ds)
    if exact_bins:
        assert np.array_equal(dev["cnt"], ref.counters)


def test_bilayer_fp64(torch_gpu, oracle_mod):
    prob = W.config0(n_primaries=5000, n_steps=120)
    dev, ref = run_both(prob, oracle_mod)
    assert_parity(dev, ref, prob)


@pytest.mark.parametrize("parallel", [True, False])
def test_spin_valve_fp32(torch_gpu, oracle_mod, parallel):
    prob = W.config1(parallel=parallel, n_primaries=7001, n_steps=160)
    dev, ref = run_both(prob, oracle_mod, slab_primaries=1024)
    assert_parity(dev, ref, prob)


def test_elastic_and_constant_tau(torch_gpu, oracle_mod):
    prob = W.homogeneous(thickness=37.5, n_primaries=3333, n_steps=90, tau0=25.0, tau_el=30.0,
                         tau_exp=0, e_edges=W.energy_edges(0.1, 2.0), state_fp64=False,
                         src=(0.0, 37.5))
    dev, ref = run_both(prob, oracle_mod, slab_primaries=700)
    assert_parity(dev, ref, prob)
    assert ref.counters[:, 2].sum() > 1000     # elastic events happened


def test_batched_instances(torch_gpu, oracle_mod):
    prob = W.config2(n_instances=6, n_steps=70, prim_lo=50, prim_hi=3000)
    prob.gen_moment = True
    dev, ref = run_both(prob, oracle_mod, slab_primaries=512)
    assert_parity(dev, ref, prob)


def test_slab_table_in_work_order(torch_gpu):
    # slabs are handed out in table order: instances by decreasing primaries per slab times
    # mean pump energy, each instance's slabs contiguous and in order
    import torch
    from paper_1807_04733_amd import PicSim
    prob = W.config2(n_instances=12, n_steps=4, prim_lo=50, prim_hi=5000)
    P = 700
    sim = PicSim(prob, slab_primaries=P)
    lay = sim.layout
    ns = lay.n_slabs
    inst = sim.ws[lay.off_slab_inst:lay.off_slab_inst + 4 * ns].view(torch.int32).cpu().numpy()
    sim.close()

    def work(it):
        S = max(1, -(-it.n_primaries // P))
        per = -(-it.n_primaries // S)
        up = it.src_up_frac
        e0 = [float(it.src_e_lo[s]) + 0.5 * float(it.src_e_span[s]) for s in (0, 1)]
        return per * (up * e0[0] + (1.0 - up) * e0[1])

    runs = [int(inst[0])] + [int(b) for a, b in zip(inst[:-1], inst[1:]) if a != b]
    assert sorted(runs) == list(range(len(prob.instances)))     # each instance contiguous
    w = [work(prob.instances[i]) for i in runs]
    assert all(x >= y for x, y in zip(w[:-1], w[1:]))
    assert runs != sorted(runs)         # the workload's instances are not already in order


def test_energy_tables_and_gaussian_pump(torch_gpu, oracle_mod):
    prob = W.config4(n_instances=3, primaries_per_instance=1500, n_steps=400)
    dev, ref = run_both(prob, oracle_mod, slab_primaries=400)
    assert_parity(dev, ref, prob)
    assert (ref.counters[:, 0] > 0).sum() > 50    # injection spread over many steps


def test_edge_cases(torch_gpu, oracle_mod):
    # an empty instance, a one-primary instance and a ragged one, single step
    insts = [W.make_instance(W.bilayer(), n_primaries=n, n_steps=1) for n in (0, 1, 65)]
    prob = W.Problem(W.with_root_offsets(insts), seed=9, dt=1.0, n_steps=1)
    dev, ref = run_both(prob, oracle_mod)
    assert_parity(dev, ref, prob)
    # no secondaries (the paper's third case)
    prob = W.config0(n_primaries=999, n_steps=60)
    prob.secondaries = False
    dev, ref = run_both(prob, oracle_mod)
    assert_parity(dev, ref, prob)


def test_results_independent_of_launch_shape(torch_gpu, oracle_mod):
    prob = W.config1(parallel=True, n_primaries=6000, n_steps=120)
    prob.dens_stride = 3
    ref = oracle_mod.run(prob)
    for tuning in ({"block": 64, "grid": 7, "compact_every": 0, "z_every": 1},
                   {"block": 128, "grid": 1000, "compact_every": 1, "compact_frac": 0.0,
                    "z_every": 8, "sub_steps": 2},
                   {"block": 256, "grid": 64, "compact_every": 5, "use_graph": 0, "z_every": 3},
                   {"block": 512, "grid": 300, "compact_every": 3, "z_every": 5,
                    "sub_steps": 2},
                   {"block": 256, "grid": 2000, "compact_every": 2, "z_every": 2,
                    "sub_steps": 2, "use_graph": 0},
                   {"block": 1024, "grid": 5, "compact_every": 4, "z_every": 4,
                    "sub_steps": 2}):
        from paper_1807_04733_amd import PicSim
        _say(f"[parity] launch shape {tuning}")
        sim = PicSim(prob, slab_primaries=1000, tuning=tuning)
        # calls of uneven length: z is written back at the end of each call
        for n in (50, 1, 6, 63):
            sim.step(n)
        dens, cur = sim.int_bins()
        cnt = sim.counters()
        sim.close()
        assert np.array_equal(dens[0], ref.dens[0])
        assert np.array_equal(cur[0], ref.cur[0])
        assert np.array_equal(cnt, ref.counters)


@pytest.mark.parametrize("cfg", ["valve", "multilayer"])
@pytest.mark.parametrize("block", [512, 1024])
def test_two_step_launches_records(torch_gpu, oracle_mod, cfg, block):
    """Two steps per launch (the common path from registers, the general path per
    sub-step), in 512- and 1024-thread workgroups (the latter with one set of histogram
    slices per CU and more queue copies beside them): per-particle records and bins equal
    the oracle's."""
    if cfg == "valve":
        prob = W.config1(parallel=False, n_primaries=5000, n_steps=121)
    else:
        prob = W.config4(n_instances=2, primaries_per_instance=1200, n_steps=251)
    prob.gen_moment = True
    dev, ref = run_both(prob, oracle_mod, slab_primaries=700,
                        tuning={"sub_steps": 2, "z_every": 4, "block": block, "grid": 16})
    assert_parity(dev, ref, prob)


@pytest.mark.parametrize("sub_steps", [1, 2])
def test_removal_at_next_event(torch_gpu, oracle_mod, sub_steps):
    """The paper's rule for the lowest energy bin (carriers below E_min removed at their
    next scattering event): records, bins and counters equal the oracle's."""
    prob = W.config1(parallel=True, n_primaries=4000, n_steps=160)
    prob.e_min_fx = W.e_fx(0.3)
    prob.absorb_next = True
    prob.gen_moment = True
    dev, ref = run_both(prob, oracle_mod, slab_primaries=900,
                        tuning={"sub_steps": sub_steps, "z_every": 4})
    assert_parity(dev, ref, prob)
    assert ref.counters[:, 5].sum() == 0          # no secondary is dropped at birth


@pytest.mark.parametrize("sub_steps", [1, 2])
def test_energy_dependent_speeds_and_rates(torch_gpu, oracle_mod, sub_steps):
    """Speeds v(E) and inelastic rates 1/tau(E) interpolated from per-channel tables
    (Fig. 1): records, bins and counters equal the oracle's, in one- and two-step
    launches."""
    prob = W.variant(W.config1(parallel=True, n_primaries=4000, n_steps=160),
                     energy_tables=True, gen_moment=True)
    dev, ref = run_both(prob, oracle_mod, slab_primaries=900,
                        tuning={"sub_steps": sub_steps, "z_every": 4})
    assert_parity(dev, ref, prob)
    assert ref.counters[:, 6].sum() > 1000        # many interface transmissions


def test_energy_tables_mixed_batch(torch_gpu, oracle_mod):
    """A batch where one instance has constant speeds (E^2 rate law) and the others
    energy tables, with energy-dependent transmission and the removal rule."""
    prob = W.variant(W.config4(n_instances=3, primaries_per_instance=1200, n_steps=300),
                     energy_tables=True, absorb_next=True)
    prob.instances[1].v_tab = prob.instances[1].r_tab = None
    prob.e_min_fx = W.e_fx(0.3)
    dev, ref = run_both(prob, oracle_mod, slab_primaries=400, tuning={"sub_steps": 2})
    assert_parity(dev, ref, prob)


@pytest.mark.parametrize("sub_steps", [1, 2])
def test_weighted_superparticles(torch_gpu, oracle_mod, sub_steps):
    """Weighted superparticles (Eq. 10) from importance sampling of the source: weights
    per record, weighted density / current / generation bins and the injected-weight
    counter equal the oracle's, in one- and two-step launches."""
    prob = W.variant(W.config1(parallel=False, n_primaries=4000, n_steps=150),
                     weights=True, gen_moment=True)
    dev, ref = run_both(prob, oracle_mod, slab_primaries=900,
                        tuning={"sub_steps": sub_steps, "z_every": 4})
    assert_parity(dev, ref, prob)
    w = ref.records["w"]
    assert w.min() != w.max()                      # the weights really differ


def test_weights_with_energy_tables_batched(torch_gpu, oracle_mod):
    """Weights together with energy-dependent channels and transmission, removal at the
    next event, over a batch where one instance has no weight table (weight 1)."""
    prob = W.variant(W.config4(n_instances=3, primaries_per_instance=1000, n_steps=240),
                     energy_tables=True, weights=True, absorb_next=True, gen_moment=True)
    prob.instances[2].w_tab = None
    prob.e_min_fx = W.e_fx(0.3)
    dev, ref = run_both(prob, oracle_mod, slab_primaries=400,
                        tuning={"sub_steps": 2, "block": 512, "grid": 3})
    assert_parity(dev, ref, prob)


@pytest.mark.parametrize("kind", ["tables", "weights", "both"])
def test_extended_modes_without_debug(torch_gpu, oracle_mod, kind):
    """The production (non-debug) kernels of the table and weight modes, in two-step
    launches with z write-back: bins, generation moment and counters equal the oracle's."""
    prob = W.variant(W.config1(parallel=True, n_primaries=5000, n_steps=120),
                     energy_tables=kind != "weights", weights=kind != "tables",
                     gen_moment=True)
    dev, ref = run_both(prob, oracle_mod, debug=False, records=False, slab_primaries=700,
                        tuning={"sub_steps": 2, "z_every": 4, "compact_every": 3,
                                "compact_frac": 0.0})
    assert_parity(dev, ref, prob)


@pytest.mark.parametrize("fp64", [False, True])
def test_compaction_every_step_records(torch_gpu, oracle_mod, fp64):
    """Compaction after every step of every slab that has a tombstone, on a workload where
    most carriers die (E_min = 0.4 eV): the live carriers above each new tail fill the
    tombstones below it, moving their weights along.  Bins and counters equal the
    oracle's, and so do the records of the live carriers (compaction drops the dead ones;
    debug runs, which keep every record, never compact)."""
    prob = W.variant(W.config1(parallel=True, n_primaries=6000, n_steps=140),
                     weights=True)
    prob.e_min_fx = W.e_fx(0.4)
    prob.state_fp64 = fp64
    dev, ref = run_both(prob, oracle_mod, debug=False, slab_primaries=300,
                        tuning={"sub_steps": 2, "z_every": 2, "compact_every": 1,
                                "compact_frac": 0.0})
    parts = dev["parts"]
    dev["parts"] = None
    assert_parity(dev, ref, prob)
    keep_d = ~parts["dead"]
    keep_r = ref.records["dead"] < 0
    live_d = {k: v[keep_d] for k, v in parts.items()}
    live_r = {k: v[keep_r] for k, v in ref.records.items()}
    assert len(live_d["uid"]) == len(live_r["uid"])
    r = compare_records(live_d, live_r, fp64, z_tol=1e-9 if fp64 else 0.0)
    _say(f"[parity] live records: joined {r['joined']} of {r['n_ref']}, match {r['frac']:.6f}")
    assert r["joined"] >= 0.999 * r["n_ref"]
    assert r["frac"] >= 0.9999, r["bad"]
    # most carriers died, and compaction removed them
    assert keep_r.sum() < 0.5 * len(ref.records["uid"])
    assert len(parts["uid"]) < 0.55 * len(ref.records["uid"])


def test_explicit_compaction_between_calls(torch_gpu, oracle_mod):
    """pic_compact between two pic_step calls (every slab with a tombstone, since
    compact_frac is 0): afterwards the slabs hold exactly their live carriers, and the
    run's bins and counters still equal the oracle's."""
    from paper_1807_04733_amd import PicSim
    prob = W.config1(parallel=False, n_primaries=5000, n_steps=100)
    prob.e_min_fx = W.e_fx(0.3)
    ref = oracle_mod.run(prob)
    sim = PicSim(prob, slab_primaries=400,
                 tuning={"compact_every": 0, "compact_frac": 0.0, "sub_steps": 2,
                         "z_every": 4})
    sim.step(37)
    before = sim.particles()
    assert before["dead"].any()
    sim.compact()
    after = sim.particles()
    assert not after["dead"].any()
    assert len(after["uid"]) == int((~before["dead"]).sum())
    assert np.array_equal(np.sort(after["uid"]), np.sort(before["uid"][~before["dead"]]))
    sim.step(63)
    dens, cur = sim.int_bins()
    cnt = sim.counters()
    sim.close()
    assert np.array_equal(dens[0], ref.dens[0])
    assert np.array_equal(cur[0], ref.cur[0])
    assert np.array_equal(cnt, ref.counters)


def test_fp64_state_with_tables_and_weights(torch_gpu, oracle_mod):
    """Binary64 particle state with energy tables and weights (records to 1e-9 nm)."""
    prob = W.variant(W.config0(n_primaries=2500, n_steps=100), energy_tables=True,
                     weights=True, gen_moment=True)
    dev, ref = run_both(prob, oracle_mod, slab_primaries=600, tuning={"sub_steps": 2})
    assert_parity(dev, ref, prob)


def test_capacity_overflow_is_reported(torch_gpu):
    from paper_1807_04733_amd import PicSim, PicError
    prob = W.config0(n_primaries=2000, n_steps=100)
    sim = PicSim(prob, capacity_factor=1.05)
    sim.step()
    with pytest.raises(PicError) as e:
        sim.counters()
    assert e.value.code == 3
    sim.close()


def test_reset_replays_identically(torch_gpu):
    from paper_1807_04733_amd import PicSim
    prob = W.config1(n_primaries=4000, n_steps=50)
    sim = PicSim(prob)
    sim.step()
    a = sim.int_bins()
    sim.reset()
    sim.step()
    b = sim.int_bins()
    sim.close()
    assert all(np.array_equal(x, y) for x, y in zip(a[0] + a[1], b[0] + b[1]))


def test_autotune_keeps_results(torch_gpu, oracle_mod):
    from paper_1807_04733_amd import PicSim
    prob = W.config2(n_instances=5, n_steps=60, prim_lo=300, prim_hi=4000)
    ref = oracle_mod.run(prob)
    sim = PicSim(prob, slab_primaries=600)
    tuned = sim.autotune(trial_steps=20)
    _say(f"[parity] autotuned {tuned}")
    assert tuned["block"] in (128, 256, 512, 1024) and tuned["grid"] > 0
    again = sim.autotune(trial_steps=20)          # served from the cache
    assert again == tuned
    sim.step()
    dens, cur = sim.int_bins()
    cnt = sim.counters()
    sim.close()
    for i in range(len(prob.instances)):
        assert np.array_equal(dens[i], ref.dens[i])
        assert np.array_equal(cur[i], ref.cur[i])
    assert np.array_equal(cnt, ref.counters)
