"""Device code paths that the standard workloads do not reach, against the oracle (GPU):
density histograms too large for LDS (global atomics), interfaces with T = 0 and T = 1,
and the error report for more than 8 boundary hits in one half step."""
import sys

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import assert_parity, run_both  # noqa: F401  (fixtures below)

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


@pytest.mark.parametrize("sub_steps", [1, 2])
def test_density_beyond_lds_uses_global_bins(torch_gpu, oracle_mod, sub_steps):
    """Fe(15)/Au(600) with 128 energy bins: the density slice (615 x 128 x 2 counters)
    does not fit in LDS, so the kernel deposits density with global atomics."""
    from paper_1807_04733_amd import PicSim
    from paper_1807_04733_amd.sim import workspace_bytes  # noqa: F401
    inst = W.make_instance(W.bilayer(15.0, 600.0), n_primaries=3000, n_steps=90,
                           e0_ev=(0.5, 0.5), e_span_ev=(1.5, 1.5))
    prob = W.Problem([inst], seed=5, dt=1.0, n_steps=90, e_edges=W.energy_edges(2.0 / 128, 2.0),
                     dens_stride=3, name="fe15_au600_128_ebins")
    assert prob.n_ebins == 128 and inst.nz == 615
    assert inst.nz * prob.n_ebins * 2 * 4 > 160 * 1024
    dev, ref = run_both(prob, oracle_mod, slab_primaries=500,
                        tuning={"sub_steps": sub_steps, "z_every": 2 * sub_steps})
    assert_parity(dev, ref, prob)
    assert ref.dens[0].sum() > 0


@pytest.mark.parametrize("T", [0.0, 1.0])
def test_interfaces_that_never_or_always_transmit(torch_gpu, oracle_mod, T):
    """T = 0 (every hit reflects, no draw) and T = 1 (every hit transmits, no draw) on an
    Fe/Au/Fe valve, records and bins equal to the oracle's."""
    inst = W.make_instance(W.spin_valve(15.0, 40.0, 15.0), n_primaries=4000, n_steps=120,
                           e0_ev=(0.5, 0.5), e_span_ev=(1.5, 1.5), T_values=(T, T, T, T))
    prob = W.Problem([inst], seed=13, dt=0.5, n_steps=120, e_edges=W.energy_edges(0.1, 2.0),
                     name=f"valve_T{T:g}")
    dev, ref = run_both(prob, oracle_mod, slab_primaries=600, tuning={"sub_steps": 2})
    assert_parity(dev, ref, prob)
    names = oracle_mod.COUNTER_NAMES
    hits = ref.counters[:, names.index("transmit")].sum() + ref.counters[:, names.index("refl_if")].sum()
    assert hits > 1000
    if T == 0.0:
        assert ref.counters[:, names.index("transmit")].sum() == 0
    else:
        assert ref.counters[:, names.index("refl_if")].sum() == 0


def test_more_than_eight_hits_is_reported(torch_gpu, oracle_mod):
    """Sixteen Au layers of 1/16 nm joined by T = 1 and half steps of up to 1 nm: a carrier
    with |cos theta| > 9/16 meets more than 8 boundaries in one half step.  The device flags
    it (PIC_ESTATE at the next synchronizing call, the kernel itself finishes normally) and
    the oracle reports its error too."""
    from paper_1807_04733_amd import PicError, PicSim
    layers = [W.Layer("Au", 1.0 / 16) for _ in range(16)]
    inst = W.make_instance(layers, n_primaries=256, n_steps=3, src_lambda=0.0,
                           tau0=(float("inf"),) * 4)
    prob = W.Problem([inst], seed=1, dt=2.0, n_steps=3, state_fp64=True, name="thin_layers")
    with pytest.raises(RuntimeError):
        oracle_mod.run(prob)
    sim = PicSim(prob)
    sim.step()
    with pytest.raises(PicError) as e:
        sim.counters()
    assert e.value.code == 5
    sim.close()
    # the same stack with half steps below one layer thickness runs clean on both sides
    ok = W.Problem([inst], seed=1, dt=0.1, n_steps=3, state_fp64=True)
    sim = PicSim(ok)
    sim.step()
    cnt = sim.counters()
    sim.close()
    assert np.array_equal(cnt, oracle_mod.run(ok).counters)


@pytest.mark.parametrize("up_frac,n", [(1.0, 150_000), (0.0, 300_000), (0.5, 200_001)])
def test_sixteen_bit_density_counters_wrap_exactly(torch_gpu, oracle_mod, up_frac, n):
    """Two-step launches whose two density slices only fit as 16-bit counters (200 depth x
    64 energy bins): one workgroup streams every carrier of one slab, and all carriers sit
    in the same cell (speed 1e-6 nm/fs, no scattering, one energy), so that a counter wraps
    several times per launch -- in the low half (spin up), the high half (spin down) or both
    with carries between them.  The int64 bins equal the oracle's exactly."""
    inf = float("inf")
    inst = W.make_instance([W.Layer("Au", 200.0)], n_primaries=n, n_steps=6,
                           v=(1e-6,) * 4, tau0=(inf,) * 4, src_lambda=0.0, up_frac=up_frac,
                           e0_ev=(1.3, 1.3))
    inst.src_z_lo = inst.src_z_hi = 100.25
    prob = W.Problem([inst], seed=2, dt=1.0, n_steps=6, e_edges=W.energy_edges(2.0 / 64, 2.0),
                     name=f"one_cell_{n}")
    from paper_1807_04733_amd import PicSim
    sim = PicSim(prob, slab_primaries=n,
                 tuning={"block": 512, "grid": 1, "sub_steps": 2, "z_every": 2,
                         "compact_every": 0})
    sim.step()
    cnt = sim.counters()
    dens, cur = sim.int_bins()
    sim.close()
    ref = oracle_mod.run(prob)
    assert np.array_equal(cnt, ref.counters)
    assert np.array_equal(dens[0], ref.dens[0])
    assert np.array_equal(cur[0], ref.cur[0])
    cell = ref.dens[0][:, 100, int(1.3 * 32)]
    assert cell.sum(axis=1).tolist() == [n] * 6
    assert cell.max() > 2 * 65536 or up_frac == 0.5


def test_slab_dead_count_is_exact(torch_gpu, oracle_mod):
    """The step kernel's per-slab dead count equals the tombstones below the slab's tail
    (the compaction takes the live count as tail - dead), after runs with and without
    compaction and with slot overflow; a compaction then leaves exactly the live carriers
    below each compacted slab's new tail."""
    import torch
    from paper_1807_04733_amd import PicSim

    def slab_state(sim):
        lay = sim.layout
        ws = sim.ws
        ns = lay.n_slabs
        sim.stream.synchronize()
        base = ws[lay.off_slab_base:lay.off_slab_base + 8 * ns].view(torch.int64).cpu().numpy()
        tail = ws[lay.off_slab_tail:lay.off_slab_tail + 4 * ns].view(torch.int32).cpu().numpy()
        dead = ws[lay.off_slab_dead:lay.off_slab_dead + 4 * ns].view(torch.int32).cpu().numpy()
        fl = ws[lay.off_flags:lay.off_flags + 4 * lay.capacity].view(torch.int32).cpu().numpy()
        live = np.array([int((fl[b:b + t] >= 0).sum()) for b, t in zip(base, tail)])
        return tail, dead, live

    for tuning, cap in (({"compact_every": 0}, 0.0), ({"compact_every": 7, "compact_frac": 0.0,
                                                     "sub_steps": 2, "z_every": 2}, 0.0),
                        ({"compact_every": 0}, 1.3)):
        prob = W.config1(parallel=False, n_primaries=6000, n_steps=90)
        sim = PicSim(prob, slab_primaries=700, tuning=tuning, capacity_factor=cap)
        sim.step(60)
        tail, dead, live = slab_state(sim)
        _say(f"[dead count] {tuning} cap {cap}: tails {tail.sum()}, dead {dead.sum()}")
        assert np.array_equal(tail - dead, live)
        if cap == 0.0:
            assert dead.sum() > 0
            sim.set_tuning(compact_frac=0.0)
            sim.compact()
            t2, d2, l2 = slab_state(sim)
            assert np.array_equal(t2, live) and np.all(d2 == 0) and np.array_equal(l2, live)
            sim.step(30)
            dens, cur = sim.int_bins()
            cnt = sim.counters()
            ref = oracle_mod.run(prob)
            assert np.array_equal(dens[0], ref.dens[0]) and np.array_equal(cnt, ref.counters)
        else:
            with pytest.raises(Exception):
                sim.counters()               # slots ran out: reported, nothing written beyond
        sim.close()


def test_default_slabs_follow_the_resident_workgroups(torch_gpu, oracle_mod):
    """Default slab size: instances of equal size get a slab count that is a multiple of
    the step kernel's resident workgroups (2 per CU); instances of different sizes get
    slabs of at most 16384 primaries.  Results stay the oracle's either way."""
    import torch
    from paper_1807_04733_amd import PicSim
    R = 2 * torch.cuda.get_device_properties(0).multi_processor_count
    one = W.config1(parallel=True, n_primaries=2_000_000, n_steps=2)
    sim = PicSim(one)
    _say(f"[slabs] one instance of 2e6 primaries: {sim.layout.n_slabs} slabs (R = {R})")
    assert sim.layout.n_slabs % R == 0
    sim.close()
    # equal instances: a multiple of R over all of them
    prob = W.config1(parallel=True, n_primaries=4000, n_steps=40)
    its = [prob.instances[0], W.make_instance(W.spin_valve(parallel=False), n_primaries=4000,
                                              n_steps=40, e0_ev=(0.5, 0.5), e_span_ev=(1.5, 1.5))]
    prob.instances = W.with_root_offsets(its)
    sim = PicSim(prob)
    n = sim.layout.n_slabs
    sim.step()
    dens, cur = sim.int_bins()
    cnt = sim.counters()
    sim.close()
    ref = oracle_mod.run(prob)
    _say(f"[slabs] two equal instances of 4000 primaries: {n} slabs")
    assert n == 2 * -(-4000 // 256)  # 256 primaries per slab at least
    for i in range(2):
        assert np.array_equal(dens[i], ref.dens[i]) and np.array_equal(cur[i], ref.cur[i])
    assert np.array_equal(cnt, ref.counters)
    # different sizes: at most 16384 primaries per slab
    big = W.config1(parallel=True, n_primaries=100_000, n_steps=2)
    its = [big.instances[0], W.make_instance(W.spin_valve(parallel=False), n_primaries=50_000,
                                             n_steps=2, e0_ev=(0.5, 0.5), e_span_ev=(1.5, 1.5))]
    big.instances = W.with_root_offsets(its)
    sim = PicSim(big)
    _say(f"[slabs] 1e5 + 5e4 primaries: {sim.layout.n_slabs} slabs")
    # 150000 / 2048 primaries per slab rounds up to the minimum of 256
    assert sim.layout.n_slabs == -(-100_000 // 256) + -(-50_000 // 256)
    sim.close()


@pytest.mark.parametrize("n_ebins", [48, 52])
def test_single_density_slice_as_16_bit_counters(torch_gpu, oracle_mod, n_ebins):
    """Two-step launches with one density slice (density every third step) on 100 depth x
    n_ebins energy bins: a 32-bit slice (38.4 or 41.6 KB) fits next to the current slices
    and the queues of a 512-thread workgroup but leaves no room for copies of queued
    carriers, a 16-bit one does (the sub-step-0 copies with 48 bins, only the sub-step-1
    head with 52), so these launches take 16-bit counters and the copies.  Counters and
    int64 bins equal the oracle's exactly."""
    layers = [W.Layer("Fe", 10.0, +1), W.Layer("Au", 90.0, 0)]
    inst = W.make_instance(layers, n_primaries=20_000, n_steps=12, e0_ev=(0.8, 2.0),
                           e_span_ev=(1.0, 0.0))
    prob = W.Problem([inst], seed=5, dt=1.0, n_steps=12, dens_stride=3,
                     e_edges=W.energy_edges(2.0 / n_ebins, 2.0), name=f"one_slice_{n_ebins}")
    assert inst.nz == 100 and prob.n_ebins == n_ebins
    from paper_1807_04733_amd import PicSim
    sim = PicSim(prob, tuning={"block": 512, "grid": 64, "sub_steps": 2, "z_every": 2,
                               "compact_every": 4})
    sim.step()
    cnt = sim.counters()
    dens, cur = sim.int_bins()
    sim.close()
    ref = oracle_mod.run(prob)
    assert np.array_equal(cnt, ref.counters)
    assert np.array_equal(dens[0], ref.dens[0])
    assert np.array_equal(cur[0], ref.cur[0])
    assert ref.dens[0].sum() > 0 and int(cnt[:, 1].sum()) > 10_000  # e-e events took place
