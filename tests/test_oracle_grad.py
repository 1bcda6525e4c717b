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
