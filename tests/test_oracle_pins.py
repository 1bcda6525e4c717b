"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every test here runs on the CPU.  The checks are closed forms, exact discrete-time
results, conservation laws, brute-force enumeration and an independent library
implementation of the random-number generator, chosen so that a dropped term, a wrong
sign or index, or a swapped operand in the oracle makes at least one of them fail.
Statistical checks use 4 standard errors estimated from the sample itself.
"""
import ctypes as C
import math
import os
import shutil
import subprocess
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
INF = float("inf")


def _run(oracle_lib, prob, **kw):
    return oracle_lib.run(prob, **kw)


def _primaries(rec):
    return (rec["uid"] >> np.uint64(32)) == 0


# --------------------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("no ROCm clang to build the rocRAND reference")
    out = str(tmp_path_factory.mktemp("ref") / "librefphilox.so")
    subprocess.run([clang, "-x", "hip", "--cuda-host-only", "-O2", "-fPIC", "-shared",
                    "-I/opt/rocm/include", "-o", out,
                    os.path.join(HERE, "pins", "rocrand_philox.cpp")], check=True)
    return C.CDLL(out)


def test_philox_matches_rocrand(oracle_lib, rocrand_ref):
    """The oracle's Philox4x32-10 equals rocRAND's engine on random counters and keys."""
    rng = np.random.default_rng(7)
    n = 2000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= (1 << 30) - 1          # the reference's offset argument holds 4*(x|y<<32)
    ctr[:8] = 0
    ctr[1, 0] = 1
    ctr[2, 3] = 0xFFFFFFFF
    for key in ([0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0x243F6A88, 0x85A308D3]):
        key = np.array(key, np.uint32)
        ref = np.zeros((n, 4), np.uint32)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        rocrand_ref.ref_philox(p(ctr), p(key), p(ref), C.c_int64(n))
        mine = np.array([oracle_lib.philox(c, key) for c in ctr])
        assert np.array_equal(mine, ref)


def test_philox_uniformity(oracle_lib):
    """chi^2 of the top byte and balance of every bit over consecutive counters."""
    words = np.array([oracle_lib.philox([i, 3, 5, 0x200], [11, 13]) for i in range(20000)],
                     np.uint32).ravel()
    counts = np.bincount(words >> 24, minlength=256)
    exp = len(words) / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert 160 < chi2 < 360                     # 255 dof, ~ +/- 4.5 sigma
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(0)
    assert np.all(np.abs(bits - 0.5) < 4 * 0.5 / math.sqrt(len(words)))


# --------------------------------------------------------------------------- A: ballistic
def _fold(u, L):
    """Reflecting-wall fold of an unfolded coordinate into [0, L]; returns (z, sign)."""
    m = np.mod(u, 2 * L)
    back = m > L
    return np.where(back, 2 * L - m, m), np.where(back, -1.0, 1.0)


def test_ballistic_homogeneous_closed_form(oracle_lib):
    """tau -> infinity: the state after n2 steps is the straight-line continuation of the
    state after n1 steps, folded by the two reflecting surfaces (Eq. 18, full reflection)."""
    Lz = 100.0

    def prob(n):
        p = W.homogeneous(thickness=Lz, n_primaries=3000, n_steps=n, tau0=INF, tau_exp=0,
                          dt=0.75, src_lambda=0.0)
        return p

    r1 = _run(oracle_lib, prob(3), records=True).records
    r2 = _run(oracle_lib, prob(211), records=True).records
    o1, o2 = np.argsort(r1["uid"]), np.argsort(r2["uid"])
    z1, mu1 = r1["z"][o1], r1["mu"][o1]
    z2, mu2 = r2["z"][o2], r2["mu"][o2]
    assert np.array_equal(r1["uid"][o1], r2["uid"][o2])
    v, t = W.V_AU, (211 - 3) * 0.75
    # unfold state 1 so that the fold below reproduces it, then fly straight
    u = z1 + v * mu1 * t
    z_exp, sgn = _fold(u, Lz)
    assert np.allclose(z2, z_exp, atol=1e-9, rtol=0)
    assert np.array_equal(np.sign(mu2), np.sign(mu1) * sgn)
    assert np.array_equal(np.abs(mu2), np.abs(mu1))
    assert np.all(r2["ev"][:, 0] == 0)


def _event_driven_flight(z, mu, layer, spin, tau, inst):
    """Exact ballistic flight over time tau by hit times, T = 1 at every interface."""
    zb = inst.z_bound
    L = len(zb) - 1
    for _ in range(10000):
        v = inst.v[inst.ch_of[layer, spin]]
        wall = zb[layer + 1] if mu > 0 else zb[layer]
        t_hit = (wall - z) / (v * mu)
        if t_hit >= tau:
            return z + v * mu * tau, mu, layer
        tau -= t_hit
        z = wall
        if mu > 0:
            if layer == L - 1:
                mu = -mu
            else:
                layer += 1
        else:
            if layer == 0:
                mu = -mu
            else:
                layer -= 1
    raise RuntimeError("too many hits")


def test_ballistic_bilayer_transparent_event_driven(oracle_lib):
    """tau -> infinity, T = 1 in a Fe/Au bilayer: the half-step transport with speed
    rescaling at the interface equals an exact flight by interface hit times."""
    def prob(n):
        inst = W.make_instance(W.bilayer(15.0, 40.0), n_primaries=1500, n_steps=n,
                               transparent=True, tau0=(INF, INF, INF, INF))
        return W.Problem([inst], seed=3, dt=1.0, n_steps=n, state_fp64=True)

    r1 = _run(oracle_lib, prob(2), records=True).records
    r2 = _run(oracle_lib, prob(90), records=True).records
    inst = prob(2).instances[0]
    o1, o2 = np.argsort(r1["uid"]), np.argsort(r2["uid"])
    for a, b in zip(o1, o2):
        z, mu, l = _event_driven_flight(r1["z"][a], r1["mu"][a], r1["layer"][a],
                                        r1["spin"][a], 88.0, inst)
        assert abs(z - r2["z"][b]) < 1e-9
        assert mu == r2["mu"][b]
        assert l == r2["layer"][b]


def _tabled(inst, v_tab, r_tab, scale):
    inst = replace(inst)
    inst.v_tab, inst.r_tab, inst.e_scale = v_tab, r_tab, scale
    return inst


def test_energy_tables_flight_interpolation_and_rate(oracle_lib):
    """Energy-dependent channels (Fig. 1 inputs).  (1) A table linear in E gives the
    linear speed at any energy: the half-step transport through a transparent Fe/Au
    interface equals an exact flight by hit times at v = a_c + b_c E.  (2) At a node energy
    the inelastic probability is 1 - exp(-dt inv_tau0 r_k): the primaries without an event
    after n steps are binomial with (1-p)^n."""
    nodes, scale = 64, 32.0                # nodes at k / 32 eV
    e = np.arange(nodes) / scale
    a = np.array([0.55, 0.25, 0.9, 0.9])
    b = np.array([0.05, 0.1, 0.2, 0.2])
    v_tab = a[:, None] + b[:, None] * e[None, :]
    r_tab = np.tile(1.0 + 0.5 * e, (4, 1))
    E0 = 1.2345                            # between nodes

    def prob(n):
        inst = W.make_instance(W.bilayer(15.0, 40.0), n_primaries=1200, n_steps=n,
                               transparent=True, tau0=(INF, INF, INF, INF), e0_ev=(E0, E0))
        return W.Problem([_tabled(inst, v_tab, r_tab, scale)], seed=5, dt=1.0, n_steps=n,
                         state_fp64=True)

    r1 = _run(oracle_lib, prob(2), records=True).records
    r2 = _run(oracle_lib, prob(80), records=True).records
    inst = replace(prob(2).instances[0])
    Efx = r1["E"][0]
    assert np.all(r1["E"] == Efx)
    inst.v = a + b * (float(Efx) * 2.0 ** -30)
    o1, o2 = np.argsort(r1["uid"]), np.argsort(r2["uid"])
    for i, j in zip(o1, o2):
        z, mu, l = _event_driven_flight(r1["z"][i], r1["mu"][i], r1["layer"][i],
                                        r1["spin"][i], 78.0, inst)
        assert abs(z - r2["z"][j]) < 1e-8
        assert mu == r2["mu"][j] and l == r2["layer"][j]
    # (2) first-event survival at a node energy
    k, n, dt, tau0, N = 40, 30, 1.0, 20.0, 20000
    hom = W.homogeneous(thickness=1e4, n_primaries=N, n_steps=n, tau0=tau0, tau_exp=0,
                        dt=dt, e0_ev=k / scale, secondaries=False, e_min_ev=0.0,
                        src=(5000.0, 5000.0))
    hom.instances[0] = _tabled(hom.instances[0], v_tab, r_tab, scale)
    rec = _run(oracle_lib, hom, records=True).records
    p = -math.expm1(-dt * (1.0 / tau0) * r_tab[2, k])
    q = (1 - p) ** n
    frac = np.mean(rec["ev"][:, 0] == 0)
    se = math.sqrt(q * (1 - q) / N)
    assert abs(frac - q) < 4 * se, (frac, q, se)


def test_interface_transmission_fraction(oracle_lib):
    """Each interface hit is an independent Bernoulli(T) draw (Sec. III.A)."""
    T = 0.3
    inst = W.make_instance(W.bilayer(15.0, 20.0), n_primaries=4000, n_steps=400,
                           T_values=(T, T, T, T), tau0=(INF, INF, INF, INF))
    res = _run(oracle_lib, W.Problem([inst], seed=5, dt=1.0, n_steps=400, state_fp64=True))
    names = oracle_lib.COUNTER_NAMES
    tr = res.counters[:, names.index("transmit")].sum()
    rf = res.counters[:, names.index("refl_if")].sum()
    n = tr + rf
    assert n > 5000
    assert abs(tr / n - T) < 4 * math.sqrt(T * (1 - T) / n)


# --------------------------------------------------------------------------- B: diffusion
def _msd_discrete(n, p, v, h):
    """Exact mean-square displacement of the split scheme after n steps of an infinite
    medium with isotropic redraws at the mid-step points (probability p each)."""
    q = 1.0 - p
    a = np.arange(2 * n)
    A, B = np.meshgrid(a, a, indexing="ij")
    lo, hi = np.minimum(A, B), np.maximum(A, B)
    k = np.maximum(0, (hi - 1) // 2 - (lo + 1) // 2 + 1)
    k = np.where(lo == hi, 0, k)
    return (v * h) ** 2 / 3.0 * np.sum(q ** k)


def _alpha_eq21(t, tau):
    e = 1.0 - math.exp(-t / tau)
    return t * e / (t - tau * e)


def test_mean_square_displacement_and_alpha(oracle_lib):
    """Elastic scattering only, infinite medium (Fig. 2 setup: 1.5 eV, tau_el = 30 fs).
    The sampled MSD matches the exact discrete-time MSD of the split scheme, and that
    MSD's generalised diffusion exponent converges to the paper's Eq. (21)."""
    dt, tau_el, v = 0.5, 30.0, W.V_AU
    p = -math.expm1(-dt / tau_el)
    msds = {}
    for n in (20, 120, 400):
        prob = W.homogeneous(thickness=2000.0, n_primaries=20000, n_steps=n, tau0=INF,
                             tau_el=tau_el, tau_exp=0, dt=dt, src=(1000.0, 1000.0))
        rec = _run(oracle_lib, prob, records=True).records
        d2 = (rec["z"] - 1000.0) ** 2
        exact = _msd_discrete(n, p, v, dt / 2)
        se = d2.std() / math.sqrt(len(d2))
        assert abs(d2.mean() - exact) < 4 * se, (n, d2.mean(), exact, se)
        assert np.all(rec["ev"][:, 3] == 0) and np.all(rec["E"] == W.e_fx(1.5))
        msds[n] = exact
    # generalised diffusion exponent of the exact discrete MSD vs Eq. (21)
    for n in (60, 200, 600):
        s0, s1 = _msd_discrete(n, p, v, dt / 2), _msd_discrete(n + 2, p, v, dt / 2)
        t = (n + 1) * dt
        alpha = t * (s1 - s0) / (2 * dt) / (0.5 * (s0 + s1))
        assert abs(alpha - _alpha_eq21(t, tau_el)) < 0.02, (n, alpha)
    assert _alpha_eq21(1e-3, tau_el) == pytest.approx(2.0, abs=1e-3)
    assert _alpha_eq21(1e5, tau_el) == pytest.approx(1.0, abs=1e-3)


def test_short_tau_diffusion_mode_decay(oracle_lib):
    """Short elastic time in a reflecting slab: the first Neumann cosine mode of the
    density decays at D (pi/L)^2 with D the diffusion constant of the discrete scheme."""
    Lz, dt, tau_el, v = 20.0, 0.25, 1.0, W.V_AU
    p = -math.expm1(-dt / tau_el)
    # D of the discrete walk from the exact MSD's linear growth
    D = (_msd_discrete(402, p, v, dt / 2) - _msd_discrete(400, p, v, dt / 2)) / (2 * 2 * dt)
    k = math.pi / Lz
    amps = []
    for n in (120, 360):
        prob = W.homogeneous(thickness=Lz, n_primaries=40000, n_steps=n, tau0=INF,
                             tau_el=tau_el, tau_exp=0, dt=dt, src=(4.0, 4.0))
        rec = _run(oracle_lib, prob, records=True).records
        c = np.cos(k * rec["z"])
        amps.append((c.mean(), c.std() / math.sqrt(len(c))))
    ratio = amps[1][0] / amps[0][0]
    expect = math.exp(-D * k * k * (360 - 120) * dt)
    err = ratio * math.hypot(amps[0][1] / amps[0][0], amps[1][1] / amps[1][0])
    assert abs(ratio - expect) < 4 * err + 0.01, (ratio, expect, err)


# --------------------------------------------------------------------------- C: cascade
def _alive_expectation(n, p, x):
    """E[N_alive] of one primary after n steps: each alive carrier splits with
    probability p per step into two carriers whose energies are E times independent
    uniforms; a carrier whose energy fraction falls below x is removed."""
    tot = 0.0
    for k in range(n + 1):
        m_k = math.comb(n, k) * (2 * p) ** k * (1 - p) ** (n - k)
        if k == 0 or x <= 0:
            surv = 1.0
        else:
            lx = -math.log(x)
            surv = 1.0 - x * sum(lx ** j / math.factorial(j) for j in range(k))
        tot += m_k * surv
    return tot


@pytest.mark.parametrize("e_min", [0.0, 0.1])
def test_cascade_closed_form(oracle_lib, e_min):
    """Constant lifetime (Fig. 3 setting): mean number of hot carriers per primary."""
    n, dt, tau = 40, 1.0, 30.0
    p = -math.expm1(-dt / tau)
    prob = W.homogeneous(thickness=60.0, n_primaries=8000, n_steps=n, tau0=tau, tau_exp=0,
                         dt=dt, e_min_ev=e_min, e0_ev=1.5)
    res = _run(oracle_lib, prob, records=True)
    rec = res.records
    alive = rec["dead"] < 0
    per_root = np.bincount((rec["uid"] & np.uint64(0xFFFFFFFF)).astype(np.int64)[alive],
                           minlength=8000)
    exp = _alive_expectation(n, p, e_min / 1.5)
    se = per_root.std() / math.sqrt(len(per_root))
    assert abs(per_root.mean() - exp) < 4 * se, (per_root.mean(), exp, se)
    assert res.counters[-1, 9] == alive.sum()


def test_mean_generation_closed_form(oracle_lib):
    """Generation map of Sec. V (mean generation label per cell), constant lifetime and
    E_min = 0: every carrier splits with probability p per step, the scattering carrier
    keeps its label and the secondary gets the label + 1, so with A_n carriers and G_n the
    sum of their labels, A_{n+1} = (1+p) A_n and G_{n+1} = (1+p) G_n + p A_n, which gives
    the mean label G_n / A_n = 1 + n p / (1+p) after n steps.  Checked on the last density
    slot (after n steps) over 8 seeds at 4 standard errors; and the per-cell moment against
    the records of the carriers alive at the end."""
    n, dt, tau = 20, 1.0, 20.0
    p = -math.expm1(-dt / tau)
    exact = 1 + n * p / (1 + p)
    vals = []
    for seed in range(8):
        prob = W.homogeneous(thickness=60.0, n_primaries=4000, n_steps=n, tau0=tau,
                             tau_exp=0, dt=dt, e_min_ev=0.0, seed=seed)
        prob.gen_moment = True
        res = _run(oracle_lib, prob, records=(seed == 0))
        vals.append(res.gen[0][-1].sum() / res.dens[0][-1].sum())
        if seed == 0:
            rec = res.records
            alive = rec["dead"] < 0
            zb = np.clip(np.floor(rec["z"][alive]).astype(int), 0, prob.instances[0].nz - 1)
            want = np.zeros((prob.instances[0].nz, 2), np.int64)
            np.add.at(want, (zb, rec["spin"][alive]), rec["gen"][alive])
            assert np.array_equal(res.gen[0][-1].astype(np.int64), want)
    m = np.mean(vals)
    se = np.std(vals, ddof=1) / math.sqrt(len(vals))
    assert abs(m - exact) < 4 * se + 1e-12, (m, exact, se)


def test_generation_moment_without_secondaries(oracle_lib):
    """Without secondaries every carrier is a primary (label 1): the generation moment is
    the density summed over energy, cell by cell."""
    prob = W.config0(n_primaries=2000, n_steps=50)
    prob.secondaries = False
    prob.gen_moment = True
    res = _run(oracle_lib, prob)
    assert np.array_equal(res.gen[0], res.dens[0].sum(axis=2))


def test_cascade_closed_form_next_scatter_removal(oracle_lib):
    """Removal at the next scattering event (Sec. III.A, lowest energy bin), constant
    lifetime: a carrier with k events in its ancestry is alive iff its energy before the
    k-th event was at least E_min (it split there; a carrier below E_min is removed at its
    event instead), i.e. E[N_alive] = sum_k m_k(n) P(prod_{i<k} U_i >= x)."""
    n, dt, tau, E0, emin = 40, 1.0, 30.0, 1.5, 0.3
    p = -math.expm1(-dt / tau)
    x = emin / E0
    exp = 0.0
    lx = -math.log(x)
    for k in range(n + 1):
        m_k = math.comb(n, k) * (2 * p) ** k * (1 - p) ** (n - k)
        surv = 1.0 if k <= 1 else 1.0 - x * sum(lx ** j / math.factorial(j) for j in range(k - 1))
        exp += m_k * surv
    prob = W.homogeneous(thickness=60.0, n_primaries=8000, n_steps=n, tau0=tau, tau_exp=0,
                         dt=dt, e_min_ev=emin, e0_ev=E0)
    prob.absorb_next = True
    res = _run(oracle_lib, prob, records=True)
    rec = res.records
    alive = rec["dead"] < 0
    per_root = np.bincount((rec["uid"] & np.uint64(0xFFFFFFFF)).astype(np.int64)[alive],
                           minlength=8000)
    se = per_root.std() / math.sqrt(len(per_root))
    assert abs(per_root.mean() - exp) < 4 * se, (per_root.mean(), exp, se)
    # the immediate-removal expectation differs by many standard errors here
    assert abs(_alive_expectation(n, p, x) - exp) > 10 * se


def test_cascade_energy_histogram(oracle_lib):
    """Energy spectrum of the cascade after n steps (E_min = 0): a carrier with k splits
    has energy E0*prod(U_i), density (ln(E0/E))^(k-1)/((k-1)! E0)."""
    n, dt, tau, E0 = 30, 1.0, 20.0, 1.6
    p = -math.expm1(-dt / tau)
    edges = W.energy_edges(0.1, 1.6)
    prob = W.homogeneous(thickness=60.0, n_primaries=6000, n_steps=n, tau0=tau, tau_exp=0,
                         dt=dt, e_min_ev=0.0, e0_ev=E0, e_edges=edges)
    res = _run(oracle_lib, prob)
    hist = res.dens[0][-1].sum(axis=(0, 2)).astype(float) / 6000
    lo = np.arange(16) * 0.1
    hi = lo + 0.1

    def cdf_k(e, k):   # P(E0 prod U <= e) for k >= 1
        x = e / E0
        if x <= 0:
            return 0.0
        lx = -math.log(x)
        return x * sum(lx ** j / math.factorial(j) for j in range(k))

    expect = np.zeros(16)
    for k in range(1, n + 1):
        m_k = math.comb(n, k) * (2 * p) ** k * (1 - p) ** (n - k)
        expect += m_k * np.array([cdf_k(b, k) - cdf_k(a, k) for a, b in zip(lo, hi)])
    expect[-1] += (1 - p) ** n          # never-split primaries sit at E0 (last bin)
    se = np.sqrt(np.maximum(expect, 1e-3) * 4 / 6000)   # generous Poisson-cluster error
    assert np.all(np.abs(hist - expect) < 4 * se + 1e-3), np.c_[hist, expect]


# --------------------------------------------------------------------------- D, E, F
@pytest.mark.parametrize("absorb_next", [False, True])
def test_conservation_counts_energy_and_bound(oracle_lib, absorb_next):
    """Integer conservation every step (Eq. 17), exact energy conservation of the
    e-e events (Sec. III.A) and the per-tree alive bound floor(E0/E_min) (immediate
    removal only: with removal at the next event, carriers below E_min stay alive)."""
    prob = W.config0(n_primaries=3000, n_steps=150)
    prob.absorb_next = absorb_next
    res = _run(oracle_lib, prob, records=True)
    c = res.counters
    names = oracle_lib.COUNTER_NAMES
    col = {k: c[:, names.index(k)] for k in names}
    net = np.cumsum(col["injected"] + col["spawned"] - col["absorbed"])
    assert np.array_equal(net, col["alive"])
    assert np.array_equal(res.dens[0].sum(axis=(1, 2, 3)).astype(np.int64), col["alive"])
    rec = res.records
    alive = rec["dead"] < 0
    e_alive = int(rec["E"][alive].astype(np.int64).sum())
    assert e_alive + int(col["e_absorbed"].sum()) == 3000 * W.e_fx(1.5)
    roots = (rec["uid"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    per_root = np.bincount(roots[alive], minlength=3000)
    if not absorb_next:
        assert per_root.max() <= W.e_fx(1.5) // prob.e_min_fx
    else:
        assert col["sec_absorbed"].sum() == 0        # every secondary is created
        assert (rec["E"][alive] < prob.e_min_fx).any()   # carriers below E_min live on
    # spawns recorded per particle add up to the spawn counter
    assert rec["ev"][:, 3].sum() == col["spawned"].sum()
    assert len(rec["uid"]) == 3000 + col["spawned"].sum()


def test_fp32_state_is_representable(oracle_lib):
    prob = W.config1(n_primaries=500, n_steps=60)
    rec = _run(oracle_lib, prob, records=True).records
    assert np.array_equal(rec["z"].astype(np.float32).astype(np.float64), rec["z"])
    assert np.array_equal(rec["mu"].astype(np.float32).astype(np.float64), rec["mu"])
    zb = prob.instances[0].z_bound
    assert np.all(rec["z"] >= zb[rec["layer"]]) and np.all(rec["z"] <= zb[rec["layer"] + 1])


# --------------------------------------------------------------------------- G: T = 1
def test_split_layer_invariance(oracle_lib):
    """Splitting a homogeneous layer into two identical layers joined by T = 1 changes
    nothing but the transmission count: the bins are bitwise identical."""
    base = dict(thickness=50.0, n_primaries=2000, n_steps=120, tau0=25.0, tau_el=40.0,
                e_min_ev=0.1, e_edges=W.energy_edges(0.25, 2.0), src=(0.0, 50.0))
    a = _run(oracle_lib, W.homogeneous(**base), records=True)
    b = _run(oracle_lib, W.homogeneous(split_at=21.0, **base), records=True)
    assert np.array_equal(a.dens[0], b.dens[0])
    assert np.array_equal(a.cur[0], b.cur[0])
    names = oracle_lib.COUNTER_NAMES
    keep = [i for i, k in enumerate(names) if k != "transmit"]
    assert np.array_equal(a.counters[:, keep], b.counters[:, keep])
    assert b.counters[:, names.index("transmit")].sum() > 100
    oa, ob = np.argsort(a.records["uid"]), np.argsort(b.records["uid"])
    assert np.array_equal(a.records["z"][oa], b.records["z"][ob])


# --------------------------------------------------------------------------- H: event trees
def test_event_tree_enumeration(oracle_lib):
    """One primary, constant tau, E_min = 0, 6 steps: the distribution of the number of
    carriers equals the exact enumeration of all split trees (chi^2)."""
    from scipy import stats
    n, dt, tau, N = 6, 1.0, 5.0, 30000
    p = -math.expm1(-dt / tau)
    dist = {1: 1.0}
    for _ in range(n):
        nxt = {}
        for m, pm in dist.items():
            for j in range(m + 1):
                pr = pm * math.comb(m, j) * p ** j * (1 - p) ** (m - j)
                nxt[m + j] = nxt.get(m + j, 0.0) + pr
        dist = nxt
    prob = W.homogeneous(thickness=40.0, n_primaries=N, n_steps=n, tau0=tau, tau_exp=0,
                         dt=dt, e_min_ev=0.0)
    rec = _run(oracle_lib, prob, records=True).records
    per_root = np.bincount((rec["uid"] & np.uint64(0xFFFFFFFF)).astype(np.int64), minlength=N)
    obs = np.bincount(per_root, minlength=65)[1:65].astype(float)
    exp = np.array([dist.get(m, 0.0) for m in range(1, 65)]) * N
    # merge the sparse tail
    cut = np.where(exp < 5)[0]
    first = cut[0] if len(cut) else len(exp)
    o = np.append(obs[:first], obs[first:].sum())
    e = np.append(exp[:first], exp[first:].sum())
    chi2 = ((o - e) ** 2 / e).sum()
    assert stats.chi2.sf(chi2, len(o) - 1) > 1e-3, (o, e)


# --------------------------------------------------------------------------- source
def test_injection_distributions(oracle_lib):
    """Primaries: depth ~ exp(-z/15 nm) truncated to the Fe layer, cos(theta) uniform,
    60 % spin up, energies uniform in [0.5, 2.0) eV (standard spin-valve pump)."""
    prob = W.config1(n_primaries=40000, n_steps=1)
    prob = replace(prob, instances=[replace(prob.instances[0],
                                            v=np.zeros(4), inv_tau0=np.zeros(4))])
    # frozen and collision-free: the records are the injected primaries
    res = _run(oracle_lib, prob, records=True)
    rec = {k: v[_primaries(res.records)] for k, v in res.records.items()}
    z = rec["z"]
    lam, d = 15.0, 15.0
    mean_exp = lam - d * math.exp(-d / lam) / (1 - math.exp(-d / lam))
    assert abs(z.mean() - mean_exp) < 4 * z.std() / math.sqrt(len(z))
    assert z.max() <= 15.0 and z.min() >= 0.0
    up = (rec["spin"] == 0).mean()
    assert abs(up - 0.6) < 4 * math.sqrt(0.24 / len(z))
    assert np.all(rec["ev"] == 0)
    E = rec["E"] / W.E_ONE
    assert E.min() >= 0.5 and E.max() < 2.0
    assert abs(E.mean() - 1.25) < 4 * E.std() / math.sqrt(len(E))
    mu = rec["mu"]
    assert abs(mu.mean()) < 4 * mu.std() / math.sqrt(len(mu))


# --------------------------------------------------------------------------- weights (Eq. 10)
def _weighted(prob, w_tab, w_scale, q_up=None):
    insts = [replace(it, w_tab=np.asarray(w_tab, np.float64), w_scale=w_scale,
                     src_up_frac=it.src_up_frac if q_up is None else q_up)
             for it in prob.instances]
    return replace(prob, instances=insts, weighted=True)


def test_unit_weights_reduce_to_counts(oracle_lib):
    """Weight 1 for every superparticle: the weighted density and generation moment are
    the counts times 2^16 and the current is the unweighted current, bin by bin; the
    injected weight is 2^16 per primary."""
    prob = W.config1(parallel=False, n_primaries=3000, n_steps=80)
    prob.gen_moment = True
    ref = _run(oracle_lib, prob)
    res = _run(oracle_lib, _weighted(prob, np.ones((2, 1)), 0.0))
    assert np.array_equal(res.dens[0], ref.dens[0] * np.uint64(65536))
    assert np.array_equal(res.gen[0], ref.gen[0] * np.uint64(65536))
    assert np.array_equal(res.cur[0], ref.cur[0])
    assert np.array_equal(res.counters, ref.counters)
    assert np.array_equal(res.counters[:, 11], 65536 * res.counters[:, 0])


def test_weights_follow_the_table_and_are_inherited(oracle_lib):
    """A primary's weight is the linear interpolation of its spin's row at its initial
    energy (checked with numpy's interp, to one unit of 2^-16 for the different rounding
    order), every secondary carries its root's weight, the injected-weight counter is the
    sum over primaries, and the density moment sums the weights of the carriers it
    counts."""
    prob = W.config1(parallel=True, n_primaries=2000, n_steps=40)
    nodes, e_max = 9, 2.0
    e = np.arange(nodes) * (e_max / (nodes - 1))
    w_tab = np.stack([0.5 + 0.7 * e, 2.0 - 0.6 * e])
    wp = _weighted(prob, w_tab, (nodes - 1) / e_max)
    res = _run(oracle_lib, wp, records=True)
    rec = res.records
    prim = _primaries(rec)
    # primaries frozen at injection: rerun with no motion and no scattering
    frozen = replace(wp, n_steps=1, instances=[replace(wp.instances[0], v=np.zeros(4),
                                                       inv_tau0=np.zeros(4))])
    f = _run(oracle_lib, frozen, records=True).records
    fp = _primaries(f)
    E0, s0, w0 = f["E"][fp] / W.E_ONE, f["spin"][fp], f["w"][fp].astype(np.int64)
    want = np.where(s0 == 0, np.interp(E0, e, w_tab[0]), np.interp(E0, e, w_tab[1]))
    assert np.abs(w0 - np.rint(want * 65536)).max() <= 1
    # inheritance: all carriers of a tree carry the root's weight
    root = (rec["uid"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    wroot = np.zeros(root.max() + 1, np.int64)
    wroot[root[prim]] = rec["w"][prim]
    assert np.array_equal(rec["w"].astype(np.int64), wroot[root])
    assert res.counters[:, 11].sum() == rec["w"][prim].astype(np.int64).sum()
    # the last density slot sums the weights of the carriers alive at the end
    alive = rec["dead"] < 0
    last = (prob.n_steps - 1) // prob.dens_stride
    if (prob.n_steps - 1) % prob.dens_stride == 0:
        assert res.dens[0][last].sum() == rec["w"][alive].astype(np.int64).sum()


def test_spin_importance_sampling_is_unbiased(oracle_lib):
    """Spin sampled 50/50 with weights p/q and (1-p)/(1-q) (p = 0.6): the weighted
    hot-carrier density per spin and the spin current agree with the unbiased unweighted
    simulation in expectation (8 seeds each, 4 standard errors of the difference), and the
    total injected weight matches the number of primaries."""
    p, q = W.SPIN_UP_FRAC, 0.5
    stats = {"plain": [], "weighted": []}
    for seed in range(8):
        prob = W.config1(parallel=False, n_primaries=3000, n_steps=60, seed=seed)
        plain = _run(oracle_lib, prob)
        wt = np.array([[p / q], [(1 - p) / (1 - q)]])
        wres = _run(oracle_lib, _weighted(replace(prob, seed=100 + seed), wt, 0.0, q_up=q))
        for name, r, scale in (("plain", plain, 1.0), ("weighted", wres, 2.0 ** -16)):
            d = r.dens[0][-1].astype(np.float64) * scale
            per_spin = d.sum(axis=(0, 1))
            js = r.cur_float(0)[-1].sum(axis=0)
            stats[name].append(np.concatenate([per_spin, js[:1] - js[1:]]))
        # E[w] = 1 and var(w) = 0.5 * 0.2^2 + 0.5 * 0.2^2 = 0.04 per primary
        assert abs(wres.counters[:, 11].sum() / 65536 - 3000) < 4 * math.sqrt(3000 * 0.04)
    a, b = np.array(stats["plain"]), np.array(stats["weighted"])
    diff = a.mean(0) - b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))
    assert np.all(np.abs(diff) < 4 * se + 1e-9), (diff, se)
    # the sampling really differs: the unweighted count of spin-up carriers moves with q
    assert b[:, 0].mean() != a[:, 0].mean()


def test_more_than_eight_hits_is_an_error(oracle_lib):
    """Sixteen Au layers of 1/16 nm joined by T = 1 and half steps of up to 1 nm: a carrier
    that would meet more than 8 boundaries in one half step makes the run fail (the limit
    of the transport loop), while half steps shorter than a layer run clean."""
    layers = [W.Layer("Au", 1.0 / 16) for _ in range(16)]
    inst = W.make_instance(layers, n_primaries=256, n_steps=3, src_lambda=0.0,
                           tau0=(INF, INF, INF, INF))
    with pytest.raises(RuntimeError):
        _run(oracle_lib, W.Problem([inst], seed=1, dt=2.0, n_steps=3, state_fp64=True))
    res = _run(oracle_lib, W.Problem([inst], seed=1, dt=0.1, n_steps=3, state_fp64=True))
    assert res.counters[:, oracle_lib.COUNTER_NAMES.index("transmit")].sum() > 0
