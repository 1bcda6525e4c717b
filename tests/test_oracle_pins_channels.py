"""Pins of the CPU oracle's per-layer channel rules and interface decisions (CPU).

Each check compares the oracle with a fact fixed by the paper or by elementary
mathematics, not with the oracle itself:
  * Eq. (19): a secondary is spin up with probability (1 + P0)/2 of the layer where it is
    lifted (P0 = +-0.2 in Fe by its magnetisation, 0 in Au) -- binomial per layer, for a
    parallel and an antiparallel valve;
  * Eq. (2) per channel: the scattering probability of a carrier uses the lifetime of the
    channel (material, spin local to the layer) -- first-event survival per layer and spin;
  * Sec. III.A interfaces: with equal speeds in both layers the free flight is a fold of
    the straight line, and each interface hit either keeps the carrier on it (transmit) or
    mirrors it about the interface with its direction reversed (reflect); the parity of the
    reflections over k hits has probability (1 + (2T - 1)^k)/2 -- per carrier to 1e-9 nm,
    by enumeration over k, for T = 0, an intermediate T and T = 1;
  * energy-dependent transmission tables: the first-hit transmitted fraction at an energy
    between two nodes equals numpy's linear interpolation of the table.
Statistical checks use 4 standard errors.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

INF = float("inf")


def _frozen(inst):
    """The same instance with every speed 0: carriers stay where they are injected."""
    return replace(inst, v=np.zeros_like(inst.v))


def _whole_stack_source(inst):
    inst = replace(inst)
    inst.src_lambda, inst.src_cd = 0.0, 0.0
    inst.src_z_lo, inst.src_z_hi = 0.0, float(inst.z_bound[-1])
    return inst


def _layer_of(inst, z):
    return np.searchsorted(inst.z_bound, z, side="right") - 1


@pytest.mark.parametrize("parallel", [True, False])
def test_secondary_spin_follows_equilibrium_polarisation(oracle_lib, parallel):
    """Frozen carriers in an Fe(15)/Au(30)/Fe(15) valve pumped over the whole stack: the
    spin-up fraction of the secondaries found in each layer is (1 + P0)/2 with P0 = +0.2 in
    the emitter, 0 in Au and +0.2 (parallel) or -0.2 (antiparallel) in the collector."""
    N, n = 8000, 40
    inst = W.make_instance(W.spin_valve(15.0, 30.0, 15.0, parallel=parallel), n_primaries=N,
                           n_steps=n, e0_ev=(1.8, 1.8))
    inst = _frozen(_whole_stack_source(inst))
    prob = W.Problem([inst], seed=11, dt=1.0, n_steps=n, state_fp64=True)
    rec = oracle_lib.run(prob, records=True).records
    sec = (rec["uid"] >> np.uint64(32)) != 0
    assert np.array_equal(rec["layer"], _layer_of(inst, rec["z"]))
    want = {0: 0.6, 1: 0.5, 2: 0.6 if parallel else 0.4}
    for layer, p in want.items():
        sel = sec & (rec["layer"] == layer)
        m = int(sel.sum())
        assert m > 2000, m
        frac = float((rec["spin"][sel] == 0).mean())
        assert abs(frac - p) < 4 * math.sqrt(p * (1 - p) / m), (layer, frac, p, m)
    # the primaries keep the pump's spin split whatever the layer
    prim = ~sec
    up = float((rec["spin"][prim] == 0).mean())
    assert abs(up - W.SPIN_UP_FRAC) < 4 * math.sqrt(0.24 / prim.sum())


@pytest.mark.parametrize("parallel", [True, False])
def test_event_probability_per_channel(oracle_lib, parallel):
    """Frozen primaries, constant lifetimes, no secondaries: the fraction without an event
    after n steps is exp(-n dt / tau0) of the channel of (layer, spin): Fe majority 20 fs,
    Fe minority 8 fs, Au 40 fs, where the spin is counted relative to the layer's
    magnetisation (an up carrier is a minority carrier in an antiparallel collector)."""
    N, n, dt = 12000, 10, 1.0
    inst = W.make_instance(W.spin_valve(15.0, 30.0, 15.0, parallel=parallel), n_primaries=N,
                           n_steps=n, up_frac=0.5)
    inst = _frozen(_whole_stack_source(inst))
    prob = W.Problem([inst], seed=4, dt=dt, n_steps=n, tau_exp=0, state_fp64=True,
                     secondaries=False, e_min_fx=0)
    rec = oracle_lib.run(prob, records=True).records
    tau = {(0, 0): 20.0, (0, 1): 8.0, (1, 0): 40.0, (1, 1): 40.0,
           (2, 0): 20.0 if parallel else 8.0, (2, 1): 8.0 if parallel else 20.0}
    for (layer, spin), t in tau.items():
        sel = (rec["layer"] == layer) & (rec["spin"] == spin)
        m = int(sel.sum())
        q = math.exp(-n * dt / t)
        frac = float((rec["ev"][sel, 0] == 0).mean())
        assert abs(frac - q) < 4 * math.sqrt(q * (1 - q) / m), (layer, spin, frac, q, m)


# ----------------------------------------------------------------- interfaces, equal speeds
def _free_fold(u, a):
    """Fold of an unfolded coordinate into [0, 2a] by the reflecting surfaces at 0 and 2a
    (period 4a); returns the position and the sign of its motion relative to u's."""
    m = np.mod(u, 4 * a)
    back = m > 2 * a
    return np.where(back, 4 * a - m, m), np.where(back, -1.0, 1.0)


def _interface_crossings(z0, u, a):
    """Number of interface hits of the free flight from z0 to u: the unfolded images of the
    interface z = a are the points a + 2 a m."""
    lo, hi = np.minimum(z0, u), np.maximum(z0, u)
    # count m with lo < a + 2am < hi
    return (np.ceil((hi - a) / (2 * a)) - np.floor((lo - a) / (2 * a)) - 1).astype(int)


@pytest.mark.parametrize("T", [0.0, 0.35, 1.0])
def test_interface_hits_fold_and_reflection_parity(oracle_lib, T):
    """tau -> infinity, Fe(8)/Au(8) with one speed in every channel and transmission T at
    the interface.  The free flight (no interface) is the fold of z0 + v mu0 t into the
    slab; each interface reflection mirrors the carrier about the interface and reverses
    its direction, a transmission leaves it on the free path.  So every carrier sits at the
    free position or its mirror image (to 1e-9 nm) with the matching direction, and over
    carriers with k interface hits the even-parity fraction is
    sum_{j even} C(k, j) (1-T)^j T^(k-j) = (1 + (2T - 1)^k)/2."""
    a, v, N, n, dt = 8.0, 1.0, 6000, 80, 0.75
    Ts = (T, T, T, T)

    def prob(speed, steps):
        inst = W.make_instance(W.bilayer(a, a), n_primaries=N, n_steps=steps, T_values=Ts,
                               tau0=(INF, INF, INF, INF), v=(speed,) * 4, src_lambda=0.0)
        return W.Problem([inst], seed=21, dt=dt, n_steps=steps, state_fp64=True)

    r0 = oracle_lib.run(prob(0.0, 1), records=True).records     # the injected state
    r1 = oracle_lib.run(prob(v, n), records=True).records
    o0, o1 = np.argsort(r0["uid"]), np.argsort(r1["uid"])
    assert np.array_equal(r0["uid"][o0], r1["uid"][o1])
    z0, mu0 = r0["z"][o0], r0["mu"][o0]
    z, mu = r1["z"][o1], r1["mu"][o1]
    u = z0 + v * mu0 * (n * dt)
    zf, sgn = _free_fold(u, a)
    k = _interface_crossings(z0, u, a)
    even = np.abs(z - zf) < 1e-9
    odd = np.abs(z - (2 * a - zf)) < 1e-9
    assert np.all(even | odd)
    clear = np.abs(zf - a) > 1e-6                   # parity readable off the position
    par = np.where(even, 0, 1)
    assert np.all(np.abs(mu) == np.abs(mu0))
    dir_free = np.sign(mu0) * sgn
    assert np.array_equal(np.sign(mu)[clear], (dir_free * (1 - 2 * par))[clear])
    # the layer bit follows the position
    assert np.array_equal(r1["layer"][o1][clear], (z[clear] > a).astype(int))
    checked = 0
    for kk in range(0, k.max() + 1):
        sel = clear & (k == kk)
        m = int(sel.sum())
        if m < 40:
            continue
        # enumerate the 2^kk transmit/reflect sequences
        p_even = sum(math.comb(kk, j) * (1 - T) ** j * T ** (kk - j) for j in range(0, kk + 1, 2))
        frac = float((par[sel] == 0).mean())
        if p_even in (0.0, 1.0):
            assert frac == p_even, (kk, frac)
        else:
            assert abs(frac - p_even) < 4 * math.sqrt(p_even * (1 - p_even) / m), (kk, frac, p_even)
        checked += 1
    assert checked >= 3 and k.max() >= 3


# ----------------------------------------------------------------- transmission tables
def _alternating_table(nodes=64, lo=0.15, hi=0.85):
    t = np.where(np.arange(nodes) % 2 == 0, lo, hi)
    t[40:] = np.linspace(0.3, 0.7, nodes - 40)       # a smooth stretch as well
    return t


def _first_hit_problem(E_ev, table, N, seed=2):
    """Fe(15)/Au(1000), carriers injected uniformly in Fe at one energy, tau -> infinity,
    45 fs: a carrier covers at most 27 nm in Fe, so it meets the interface at most once,
    and a transmitted carrier never comes back from the thick Au layer."""
    tabs = np.stack([table] * 4)
    inst = W.make_instance(W.bilayer(15.0, 1000.0), n_primaries=N, n_steps=45,
                           T_tables=tabs, T_emax=2.0, tau0=(INF, INF, INF, INF),
                           e0_ev=(E_ev, E_ev), src_lambda=0.0, dz=5.0)
    return W.Problem([inst], seed=seed, dt=1.0, n_steps=45, state_fp64=True)


ENERGY_CASES = [(3, 0.25), (8, 0.5), (21, 0.8), (45, 0.4)]   # (node k, fraction f)


@pytest.mark.parametrize("k,f", ENERGY_CASES)
def test_transmission_table_first_hit_fraction(oracle_lib, k, f):
    """Energy-dependent transmission (64 nodes on 0-2 eV): at an energy between nodes k and
    k+1 the fraction of first interface hits that transmit is np.interp of the table."""
    table = _alternating_table()
    E = (k + f) * 2.0 / 63
    prob = _first_hit_problem(E, table, 16000)
    res = oracle_lib.run(prob)
    names = oracle_lib.COUNTER_NAMES
    tr = int(res.counters[:, names.index("transmit")].sum())
    rf = int(res.counters[:, names.index("refl_if")].sum())
    nh = tr + rf
    Efx = int(prob.instances[0].src_e_lo[0])
    nodes = np.arange(64) * (2.0 / 63)
    want = float(np.interp(Efx * 2.0 ** -30, nodes, table))
    assert nh > 5000
    assert abs(tr / nh - want) < 4 * math.sqrt(want * (1 - want) / nh), (tr / nh, want, nh)


# ----------------------------------------------------------------- one step, by hand
def test_one_step_kinematics_of_a_split(oracle_lib):
    """One step in a thick slab (no boundary reached), constant lifetime, E_min = 0.  Strang
    order (Eq. 15): a half-step flight from the injected state, the event at the mid-step
    point, then a half-step flight of the scattered carrier and of its secondary from that
    point.  Per tree with a split: both final positions are z_mid + v mu' h with their own
    final directions (to 1e-12 nm), the energies add up to the primary's exactly (Sec.
    III.A), the secondary carries generation 2.  Random-k (Eq. 4): the two new directions
    are independent and uniform -- their correlation over trees is 0 and their means 0
    within 4 standard errors; the kept energy fraction E1/E0 is uniform (Eq. 7)."""
    from scipy import stats
    N, dt, v, tau = 20000, 1.0, W.V_AU, 0.7
    h = 0.5 * dt

    def prob(speed, t):
        p = W.homogeneous(thickness=400.0, n_primaries=N, n_steps=1, tau0=t, tau_exp=0,
                          dt=dt, e_min_ev=0.0, src=(200.0, 200.0), seed=17)
        p.instances[0] = replace(p.instances[0], v=np.full(4, speed))
        return p

    r0 = oracle_lib.run(prob(0.0, INF), records=True).records     # the injected state
    r1 = oracle_lib.run(prob(v, tau), records=True).records
    prim0 = (r0["uid"] >> np.uint64(32)) == 0
    root0 = (r0["uid"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    z0 = np.zeros(N)
    mu0 = np.zeros(N)
    E0 = np.zeros(N, np.int64)
    z0[root0[prim0]] = r0["z"][prim0]
    mu0[root0[prim0]] = r0["mu"][prim0]
    E0[root0[prim0]] = r0["E"][prim0]
    root = (r1["uid"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    sec = (r1["uid"] >> np.uint64(32)) != 0
    assert np.all(r1["gen"][sec] == 2) and np.all(r1["gen"][~sec] == 1)
    p_idx = np.full(N, -1)
    c_idx = np.full(N, -1)
    p_idx[root[~sec]] = np.nonzero(~sec)[0]
    c_idx[root[sec]] = np.nonzero(sec)[0]
    split = c_idx >= 0
    n_split = int(split.sum())
    p_ev = 1.0 - math.exp(-dt / tau)
    assert abs(n_split / N - p_ev) < 4 * math.sqrt(p_ev * (1 - p_ev) / N)
    zmid = z0 + v * mu0 * h
    pi, ci = p_idx[split], c_idx[split]
    mp, mc = r1["mu"][pi], r1["mu"][ci]
    assert np.allclose(r1["z"][pi], zmid[split] + v * mp * h, rtol=0, atol=1e-12)
    assert np.allclose(r1["z"][ci], zmid[split] + v * mc * h, rtol=0, atol=1e-12)
    # no event: the straight flight of a whole step, direction kept
    keep = ~split
    assert np.allclose(r1["z"][p_idx[keep]], z0[keep] + v * mu0[keep] * dt, rtol=0, atol=1e-12)
    assert np.array_equal(r1["mu"][p_idx[keep]], mu0[keep])
    assert np.array_equal(r1["E"][pi].astype(np.int64) + r1["E"][ci], E0[split])
    se = 4.0 / math.sqrt(n_split)
    assert abs(np.corrcoef(mp, mc)[0, 1]) < se
    assert abs(np.corrcoef(mp, mu0[split])[0, 1]) < se
    assert abs(mp.mean()) < se / math.sqrt(3) and abs(mc.mean()) < se / math.sqrt(3)
    frac = r1["E"][pi] / E0[split]
    assert stats.kstest(frac, "uniform").pvalue > 1e-3


def test_density_bins_are_lower_edge_inclusive(oracle_lib):
    """Moments of Eq. (16) binned as [edge_k, edge_(k+1)) in energy and [k dz, (k+1) dz) in
    depth: the last density slot equals numpy's histogram of the records of the carriers
    alive at the end, for a pump whose energy lies exactly on a bin edge (1.5 eV with
    0.1 eV bins) and carriers that keep it (no scattering)."""
    edges = W.energy_edges(0.1, 2.0)
    inst = W.make_instance(W.bilayer(15.0, 40.0), n_primaries=3000, n_steps=25,
                           e0_ev=(1.5, 1.5), tau0=(INF, INF, INF, INF))
    prob = W.Problem([inst], seed=8, dt=1.0, n_steps=25, state_fp64=True, e_edges=edges)
    assert W.e_fx(1.5) in set(int(e) for e in edges)
    res = oracle_lib.run(prob, records=True)
    rec = res.records
    alive = rec["dead"] < 0
    zb = np.clip(np.floor(rec["z"][alive] * inst.inv_dz).astype(int), 0, inst.nz - 1)
    eb = np.clip(np.digitize(rec["E"][alive], edges.astype(np.float64), right=False) - 1, 0, None)
    want = np.zeros((inst.nz, len(edges), 2), np.int64)
    np.add.at(want, (zb, eb, rec["spin"][alive]), 1)
    assert np.array_equal(res.dens[0][-1].astype(np.int64), want)
    assert want[:, 15].sum() == alive.sum()
