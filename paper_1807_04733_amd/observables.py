"""Observables of Sec. V of arXiv:1807.04733 computed from the binned moments.

All functions take the per-instance bins as returned by `PicSim.deposit()` /
`PicSim.generations()` (torch tensors or numpy arrays) and return numpy arrays:

* density  dens[slot, z, E, spin]  carriers per cell (Eq. 16),
* current  cur[slot, z, spin]      sum of v cos(theta) per cell, nm/fs (Eq. 23 moment),
* gen      gen[slot, z, spin]      sum of generation labels per density cell.

With weighted superparticles (Eq. 10) every moment is a sum of weights, and
`normalization` gives the constant C that scales them to the excitation density.

Time slot n holds the moments after n+1 steps (t = (n+1) dt, times the stride).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np


def _np(a) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a, dtype=np.float64)


def normalization(counters, rho_exc: float) -> float:
    """The constant C of Eq. (10), rho_exc / sum_i w_i, taken over the primaries (the
    excitation that rho_exc describes): the injected-weight counter holds sum w in 2^-16
    units.  Multiplying a (weighted) density or current moment by C turns it into a
    density of the excitation rho_exc.  `counters` is one instance's [n_steps, NC] array
    (a batch of instances shares the counters, so use it with a single instance)."""
    w = float(np.asarray(counters)[:, 11].sum()) * 2.0 ** -16
    return rho_exc / w if w > 0 else 0.0


def hot_density(dens) -> np.ndarray:
    """n_hot[slot, z, spin]: the density summed over energy."""
    return _np(dens).sum(axis=2)


def depth_mask(nz: int, dz: float, z_lo: float, z_hi: float) -> np.ndarray:
    """Depth bins whose centres lie in [z_lo, z_hi) (bins of width dz from z = 0)."""
    zc = (np.arange(nz) + 0.5) * dz
    return (zc >= z_lo) & (zc < z_hi)


def p_hot(dens, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Hot-carrier spin polarisation, Eq. (22): (n_up - n_down) / (n_up + n_down).

    Per (slot, z) cell, or with a depth mask the polarisation of the carriers summed over
    those bins (a layer average as in Figs. 4 and 6) per slot.  NaN where no carrier is."""
    n = hot_density(dens)
    if mask is not None:
        n = n[:, np.asarray(mask, bool), :].sum(axis=1)
    up, dn = n[..., 0], n[..., 1]
    tot = up + dn
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(tot > 0, (up - dn) / np.where(tot > 0, tot, 1.0), np.nan)


def spin_current(cur, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Spin-current moment, Eq. (23) with the charge dropped: J_up - J_down per (slot, z)
    in nm/fs per bin, or summed over a depth mask per slot."""
    c = _np(cur)
    js = c[..., 0] - c[..., 1]
    if mask is not None:
        js = js[:, np.asarray(mask, bool)].sum(axis=1)
    return js


def mean_generation(gen, dens, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Mean generation label per (slot, z) cell (Figs. 5 and 7; 1 = primaries only), or
    over a depth mask per slot.  NaN where no carrier is."""
    g = _np(gen).sum(axis=2)
    n = hot_density(dens).sum(axis=2)
    if mask is not None:
        m = np.asarray(mask, bool)
        g, n = g[:, m].sum(axis=1), n[:, m].sum(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(n > 0, g / np.where(n > 0, n, 1.0), np.nan)


def mean_square_displacement(dens, dz: float, z0: float, sheppard: bool = True) -> np.ndarray:
    """sigma^2(t) = <(z - z0)^2> over the carriers, per slot, from the depth histogram with
    bin centres; `sheppard` adds dz^2/12, the variance of a position uniform in its bin."""
    n = hot_density(dens).sum(axis=2)
    zc = (np.arange(n.shape[1]) + 0.5) * dz
    tot = n.sum(axis=1)
    m2 = (n * (zc - z0) ** 2).sum(axis=1) / np.where(tot > 0, tot, 1.0)
    return m2 + (dz * dz / 12.0 if sheppard else 0.0)


def alpha(msd: Sequence[float], t: Sequence[float]) -> np.ndarray:
    """Generalised diffusion exponent of Sec. IV, alpha = t / sigma^2 d sigma^2 / dt, with
    the derivative taken as the centred difference of ln sigma^2 over ln t (one-sided at
    the ends)."""
    s = np.log(np.asarray(msd, dtype=np.float64))
    lt = np.log(np.asarray(t, dtype=np.float64))
    return np.gradient(s, lt)


def alpha_ballistic_diffusive(t, tau: float) -> np.ndarray:
    """The continuum result for isotropic elastic scattering with lifetime tau (Sec. IV):
    alpha(t) = t (1 - e^{-t/tau}) / (t - tau (1 - e^{-t/tau})), from 2 (ballistic) to 1."""
    t = np.asarray(t, dtype=np.float64)
    e = -np.expm1(-t / tau)
    return t * e / (t - tau * e)
