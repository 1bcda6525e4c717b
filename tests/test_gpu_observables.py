"""Observables of Sec. IV-V from the GPU's bins (needs an MI355X): the generalised
diffusion exponent of the elastic-only infinite medium against the exact discrete MSD
and the continuum formula."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from paper_1807_04733_amd import observables as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _msd_discrete(n, p, v, h):
    q = 1.0 - p
    a = np.arange(2 * n)
    A, B = np.meshgrid(a, a, indexing="ij")
    lo, hi = np.minimum(A, B), np.maximum(A, B)
    k = np.maximum(0, (hi - 1) // 2 - (lo + 1) // 2 + 1)
    k = np.where(lo == hi, 0, k)
    return (v * h) ** 2 / 3.0 * np.sum(q ** k)


def test_alpha_of_elastic_transport(torch_gpu):
    from paper_1807_04733_amd import PicSim
    dt, tau, v, n, N = 1.0, 30.0, W.V_AU, 200, 4_000_000
    p = -math.expm1(-dt / tau)
    prob = W.homogeneous(thickness=1000.0, n_primaries=N, n_steps=n, tau0=float("inf"),
                         tau_el=tau, tau_exp=0, dt=dt, src=(500.0, 500.0), state_fp64=False)
    print(f"[observables] elastic infinite medium, {N} primaries, {n} steps", file=sys.stderr,
          flush=True)
    sim = PicSim(prob, capacity_factor=1.1)
    sim.step()
    sim.counters()
    dens, _ = sim.deposit()
    sim.close()
    msd = O.mean_square_displacement(dens[0], 1.0, 500.0)
    exact = np.array([_msd_discrete(k + 1, p, v, dt / 2) for k in range(n)])
    # four standard errors of a mean of (z - z0)^2 (about sqrt(2) * MSD / sqrt(N))
    tol = 4 * math.sqrt(2.0) * exact / math.sqrt(N) + 0.05
    assert np.all(np.abs(msd[9:] - exact[9:]) < tol[9:])
    t = (np.arange(n) + 1) * dt
    a = O.alpha(msd, t)
    c = O.alpha_ballistic_diffusive(t, tau)
    sel = (t >= 30) & (t <= 180)
    assert np.max(np.abs(a[sel] - c[sel])) < 0.03, np.max(np.abs(a[sel] - c[sel]))
