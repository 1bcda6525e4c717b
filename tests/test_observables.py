"""Observables of Sec. V from the binned moments (CPU, on the oracle's bins): checked
against the per-particle records of the same run and against closed forms."""
import math

import numpy as np

import workloads as W
from paper_1807_04733_amd import observables as O


def _alive_last(rec):
    return rec["dead"] < 0


def test_p_hot_current_and_generation_match_records(oracle_lib):
    """Last density slot: per-cell P_hot (Eq. 22), a layer average, the spin-current moment
    (Eq. 23) and the mean generation computed from the bins equal the same quantities
    computed directly from the records of the carriers alive at the end."""
    prob = W.config0(n_primaries=3000, n_steps=80)
    prob.gen_moment = True
    res = oracle_lib.run(prob, records=True)
    inst = prob.instances[0]
    rec = res.records
    a = _alive_last(rec)
    zb = np.clip(np.floor(rec["z"][a] * inst.inv_dz).astype(int), 0, inst.nz - 1)
    s = rec["spin"][a]
    n = np.zeros((inst.nz, 2))
    np.add.at(n, (zb, s), 1.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        want = (n[:, 0] - n[:, 1]) / (n[:, 0] + n[:, 1])
    got = O.p_hot(res.dens[0])[-1]
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.allclose(got[ok], want[ok], rtol=0, atol=1e-15)
    # Fe layer average (the first 15 nm)
    fe = O.depth_mask(inst.nz, 1.0 / inst.inv_dz, 0.0, 15.0)
    nu, nd = n[fe, 0].sum(), n[fe, 1].sum()
    assert O.p_hot(res.dens[0], fe)[-1] == (nu - nd) / (nu + nd)
    # spin current from the records: v(layer, spin) * cos(theta) summed per bin
    v = np.array([[inst.v[inst.ch_of[l][sp]] for sp in (0, 1)] for l in range(inst.n_layers)])
    vm = v[rec["layer"][a], s] * rec["mu"][a]
    js = np.zeros(inst.nz)
    np.add.at(js, zb, np.where(s == 0, vm, -vm))
    got_js = O.spin_current(res.cur_float(0))[-1]
    assert np.allclose(got_js, js, rtol=0, atol=1e-6)
    # mean generation
    g = np.zeros(inst.nz)
    np.add.at(g, zb, rec["gen"][a])
    tot = n.sum(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        want_g = g / tot
    got_g = O.mean_generation(res.gen[0], res.dens[0])[-1]
    ok = tot > 0
    assert np.allclose(got_g[ok], want_g[ok], rtol=0, atol=1e-12)
    assert np.all(np.isnan(got_g[~ok]))


def _msd_discrete(n, p, v, h):
    """Exact MSD of the split scheme with isotropic redraws at the mid-step points
    (probability p each) after n steps: (vh)^2/3 times the sum over pairs of half steps of
    (1-p)^(events between them)."""
    q = 1.0 - p
    a = np.arange(2 * n)
    A, B = np.meshgrid(a, a, indexing="ij")
    lo, hi = np.minimum(A, B), np.maximum(A, B)
    k = np.maximum(0, (hi - 1) // 2 - (lo + 1) // 2 + 1)
    k = np.where(lo == hi, 0, k)
    return (v * h) ** 2 / 3.0 * np.sum(q ** k)


def test_msd_and_alpha_from_bins(oracle_lib):
    """Elastic scattering only in an infinite medium (the Sec. IV / Fig. 2 setting): the MSD
    from the depth histogram (bin centres + dz^2/12) matches the exact discrete MSD, and
    the exponent alpha extracted from the exact MSD sequence approaches the continuum
    formula of Sec. IV (within 0.02 from t = 30 fs)."""
    dt, tau, v = 1.0, 30.0, W.V_AU
    p = -math.expm1(-dt / tau)
    n = 120
    prob = W.homogeneous(thickness=1000.0, n_primaries=20000, n_steps=n, tau0=float("inf"),
                         tau_el=tau, tau_exp=0, dt=dt, src=(500.0, 500.0))
    res = oracle_lib.run(prob)
    msd = O.mean_square_displacement(res.dens[0], 1.0, 500.0)
    for k in (19, 59, 119):
        exact = _msd_discrete(k + 1, p, v, dt / 2)
        # standard error of a mean of (z - z0)^2: about sqrt(2) * exact / sqrt(N)
        assert abs(msd[k] - exact) < 4 * math.sqrt(2.0) * exact / math.sqrt(20000) + 0.2, (k, msd[k], exact)
    t = np.arange(1, 301) * dt
    exact = np.array([_msd_discrete(k, p, v, dt / 2) for k in range(1, 301)])
    a = O.alpha(exact, t)
    c = O.alpha_ballistic_diffusive(t, tau)
    sel = t >= 30
    assert np.max(np.abs(a[sel][:-1] - c[sel][:-1])) < 0.02
    assert abs(O.alpha_ballistic_diffusive(np.array([1e-3]), tau)[0] - 2.0) < 1e-3
    assert abs(O.alpha_ballistic_diffusive(np.array([1e5]), tau)[0] - 1.0) < 1e-3


def test_normalization_constant(oracle_lib):
    """C of Eq. (10) is rho_exc over the summed primary weights: the number of primaries
    without weights, the sum of the primaries' record weights with them."""
    prob = W.config1(parallel=False, n_primaries=1500, n_steps=30)
    res = oracle_lib.run(prob)
    assert O.normalization(res.counters, 3.0) == 3.0 / 1500
    wp = W.variant(prob, weights=True)
    res = oracle_lib.run(wp, records=True)
    prim = (res.records["uid"] >> np.uint64(32)) == 0
    wsum = res.records["w"][prim].astype(np.float64).sum() * 2.0 ** -16
    assert abs(O.normalization(res.counters, 3.0) * wsum / 3.0 - 1.0) < 1e-15
