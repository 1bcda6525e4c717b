"""Pins of the oracle's likelihood-ratio gradient (CPU).

Checks: the derivative of a closed-form cascade expectation, a loss whose expectation
does not depend on the parameters (zero-mean score), and common-random-number central
finite differences of the oracle itself for a transmission node.  Each statistical check
uses 4 standard errors over independent seeds.
"""
import math

import numpy as np
import pytest

import workloads as W


def _seeds(fn, n):
    vals = np.array([fn(s) for s in range(n)])
    return vals.mean(axis=0), vals.std(axis=0, ddof=1) / math.sqrt(n)


@pytest.mark.parametrize("per_tree", [False, True])
def test_gradient_of_cascade_closed_form(oracle_lib, per_tree):
    """Constant tau, E_min = 0, no interfaces: E[N_alive after n steps] = (1+p)^n per
    primary, so d/d ln tau0 = n (1+p)^(n-1) * (-x e^-x) with x = dt/tau0."""
    n, dt, tau, N = 20, 1.0, 20.0, 6000
    x = dt / tau
    p = -math.expm1(-x)
    exact = n * (1 + p) ** (n - 1) * (-x * math.exp(-x))

    def one(seed):
        prob = W.homogeneous(thickness=60.0, n_primaries=N, n_steps=n, tau0=tau, tau_exp=0,
                             dt=dt, e_min_ev=0.0, seed=seed)
        gd = np.zeros(prob.dens_shape(0))
        gd[-1] = 1.0
        g = oracle_lib.run(prob, g_dens=[gd], grad_per_tree=per_tree).grad
        return (g[W.AU_UP] + g[W.AU_DN]) / N

    m, se = _seeds(one, 10)
    assert abs(m - exact) < 4 * se + 1e-3, (m, exact, se)


@pytest.mark.parametrize("per_tree", [False, True])
def test_gradient_with_next_scatter_removal(oracle_lib, per_tree):
    """Removal at the next event with E_min > 0, constant tau: E[N_alive after n steps] =
    sum_k m_k(n, p) P_k with m_k = C(n,k) (2p)^k (1-p)^(n-k) and P_k = P(prod_{i<k} U_i >=
    x) independent of tau0, so d/d ln tau0 = sum_k m_k (k/p - (n-k)/(1-p)) P_k dp/d ln tau0
    with dp/d ln tau0 = -x_dt e^{-x_dt}, x_dt = dt/tau0."""
    n, dt, tau, E0, emin, N = 20, 1.0, 20.0, 1.5, 0.3, 6000
    xd = dt / tau
    p = -math.expm1(-xd)
    x = emin / E0
    lx = -math.log(x)
    dsum = 0.0
    for k in range(n + 1):
        m_k = math.comb(n, k) * (2 * p) ** k * (1 - p) ** (n - k)
        P_k = 1.0 if k <= 1 else 1.0 - x * sum(lx ** j / math.factorial(j) for j in range(k - 1))
        dsum += m_k * (k / p - (n - k) / (1 - p)) * P_k
    exact = dsum * (-xd * math.exp(-xd))

    def one(seed):
        prob = W.homogeneous(thickness=60.0, n_primaries=N, n_steps=n, tau0=tau, tau_exp=0,
                             dt=dt, e_min_ev=emin, e0_ev=E0, seed=seed)
        prob.absorb_next = True
        gd = np.zeros(prob.dens_shape(0))
        gd[-1] = 1.0
        g = oracle_lib.run(prob, g_dens=[gd], grad_per_tree=per_tree).grad
        return (g[W.AU_UP] + g[W.AU_DN]) / N

    m, se = _seeds(one, 10)
    assert abs(m - exact) < 4 * se + 1e-3, (m, exact, se)


def test_zero_mean_score(oracle_lib):
    """Without secondaries and without absorption the number of carriers is the number
    injected whatever tau0 and T are: the gradient estimate has zero mean."""
    def one(seed):
        prob = W.config0(n_primaries=3000, n_steps=40, seed=seed)
        prob.secondaries = False
        prob.e_min_fx = 0
        gd = np.ones(prob.dens_shape(0))
        g = oracle_lib.run(prob, g_dens=[gd]).grad
        return g / 3000

    m, se = _seeds(one, 8)
    assert np.all(np.abs(m) <= 4 * se + 1e-12), (m, se)


@pytest.mark.parametrize("per_tree", [False, True])
def test_transmission_gradient_vs_crn_differences(oracle_lib, per_tree):
    """d/dT of the carriers found in Au after 60 fs: the likelihood-ratio estimate agrees
    with central differences taken on common random numbers."""
    h, N, n = 0.02, 6000, 60

    def prob_for(T, seed):
        inst = W.make_instance(W.bilayer(15.0, 40.0), n_primaries=N, n_steps=n,
                               T_values=(T, 0.4, T, 0.4))
        return W.Problem([inst], seed=seed, dt=1.0, n_steps=n, state_fp64=True)

    def loss_weights(prob):
        gd = np.zeros(prob.dens_shape(0))
        gd[-1, 15:] = 1.0          # Au bins of the last step
        return gd

    def lr(seed):
        prob = prob_for(0.8, seed)
        g = oracle_lib.run(prob, g_dens=[loss_weights(prob)], grad_per_tree=per_tree).grad
        # nodes of the Fe->Au and Au->Fe majority tables (the same value T)
        C = prob.instances[0].n_channels
        return (g[C + W.T_FEAU_MAJ] + g[C + W.T_AUFE_MAJ]) / N

    def fd(seed):
        vals = []
        for T in (0.8 + h, 0.8 - h):
            prob = prob_for(T, seed)
            res = oracle_lib.run(prob)
            vals.append((res.dens[0][-1, 15:].sum()) / N)
        return (vals[0] - vals[1]) / (2 * h)

    m_lr, se_lr = _seeds(lr, 8)
    m_fd, se_fd = _seeds(fd, 8)
    assert abs(m_lr - m_fd) < 4 * math.hypot(se_lr, se_fd), (m_lr, se_lr, m_fd, se_fd)
    assert abs(m_fd) > 4 * se_fd          # the derivative is resolved at all


@pytest.mark.parametrize("per_tree", [False, True])
def test_gradient_with_elastic_channel_closed_form(oracle_lib, per_tree):
    """Constant lifetimes with an elastic channel (tau_el = 30 fs, Eq. 8) and E_min = 0.  A
    step splits a carrier with probability p q: p = 1 - exp(-x), x = dt (1/tau0 + 1/tau_el)
    (Eq. 2), and q = (1/tau0) / (1/tau0 + 1/tau_el) the inelastic share of the events
    (Eq. 5); an elastic event only turns the carrier.  So E[N_alive after n steps] =
    (1 + p q)^n per primary and d/d ln tau0 = n (1 + p q)^(n-1) d(pq)/d ln tau0, with
    dp/d ln tau0 = -x_in e^-x (x_in = dt / tau0) and dq/d ln tau0 = q (q - 1)."""
    n, dt, tau, tel, N = 20, 1.0, 20.0, 30.0, 6000
    x_in, x = dt / tau, dt * (1.0 / tau + 1.0 / tel)
    p = -math.expm1(-x)
    q = (1.0 / tau) / (1.0 / tau + 1.0 / tel)
    dpq = q * (-x_in * math.exp(-x)) + p * q * (q - 1.0)
    exact = np.array([(1 + p * q) ** n, n * (1 + p * q) ** (n - 1) * dpq])

    def one(seed):
        prob = W.homogeneous(thickness=60.0, n_primaries=N, n_steps=n, tau0=tau, tau_el=tel,
                             tau_exp=0, dt=dt, e_min_ev=0.0, seed=seed)
        gd = np.zeros(prob.dens_shape(0))
        gd[-1] = 1.0
        res = oracle_lib.run(prob, g_dens=[gd], grad_per_tree=per_tree)
        g = res.grad
        return [res.counters[-1, 9] / N, (g[W.AU_UP] + g[W.AU_DN]) / N]

    m, se = _seeds(one, 10)
    assert np.all(np.abs(m - exact) < 4 * se), (m, exact, se)
    # the elastic events happen at the expected share of all events
    prob = W.homogeneous(thickness=60.0, n_primaries=N, n_steps=n, tau0=tau, tau_el=tel,
                         tau_exp=0, dt=dt, e_min_ev=0.0, seed=99)
    c = oracle_lib.run(prob).counters
    ee, el = c[:, 1].sum(), c[:, 2].sum()
    assert abs(el / (ee + el) - (1 - q)) < 4 * math.sqrt(q * (1 - q) / (ee + el))


def _first_hit_problem(E_ev, table, N, seed):
    """Fe(15)/Au(1000), carriers injected uniformly in Fe at one energy, tau -> infinity,
    45 fs: a carrier covers at most 27 nm in Fe, so it meets the interface at most once,
    and a transmitted carrier never comes back from the thick Au layer."""
    inf = float("inf")
    inst = W.make_instance(W.bilayer(15.0, 1000.0), n_primaries=N, n_steps=45,
                           T_tables=np.stack([table] * 4), T_emax=2.0,
                           tau0=(inf, inf, inf, inf), e0_ev=(E_ev, E_ev), src_lambda=0.0,
                           dz=5.0)
    return W.Problem([inst], seed=seed, dt=1.0, n_steps=45, state_fp64=True)


@pytest.mark.parametrize("per_tree", [False, True])
@pytest.mark.parametrize("k,f", [(8, 0.25), (45, 0.6)])
def test_transmission_table_gradient_split_between_nodes(oracle_lib, per_tree, k, f):
    """64-node transmission tables, carriers that meet the interface at most once (one
    energy between nodes k and k+1, weights 1-f and f): the expected number of carriers in
    Au at the end is N_hit T(E) with T(E) = (1-f) T_k + f T_(k+1), and N_hit, the number of
    first hits, does not depend on T.  So the gradient is N_hit (1-f) on node k and
    N_hit f on node k+1 (summed over the Fe->Au tables of both spins) and exactly 0 on
    every other node and on the Au->Fe tables.  The estimate's standard error per hit is
    w sqrt(1/T - 1)."""
    table = 0.5 + 0.3 * np.sin(np.arange(64) * 1.7)
    prob = _first_hit_problem((k + f) * 2.0 / 63, table, 12000, seed=3)
    gd = np.zeros(prob.dens_shape(0))
    gd[-1, 3:] = 1.0                        # depth bins of Au (5 nm each, Au from 15 nm)
    res = oracle_lib.run(prob, g_dens=[gd], grad_per_tree=per_tree)
    names = oracle_lib.COUNTER_NAMES
    nh = int(res.counters[:, names.index("transmit")].sum() +
             res.counters[:, names.index("refl_if")].sum())
    assert nh > 4000
    C = prob.instances[0].n_channels
    g = res.grad[C:].reshape(4, 64)
    x = float(prob.instances[0].src_e_lo[0]) * 2.0 ** -30 * (63 / 2.0)
    fr = x - math.floor(x)
    T = table[k] + (table[k + 1] - table[k]) * fr
    for node, w in ((k, 1.0 - fr), (k + 1, fr)):
        got = g[0, node] + g[1, node]
        se = w * math.sqrt(nh * (1.0 / T - 1.0))
        assert abs(got - nh * w) < 4 * se, (node, got, nh * w, se)
    mask = np.ones((4, 64), bool)
    mask[:2, [k, k + 1]] = False
    assert np.all(g[mask] == 0.0)
    assert np.all(res.grad[:C] == 0.0)      # nothing scatters
