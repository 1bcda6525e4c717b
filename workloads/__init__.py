"""Seeded synthetic workloads for the spin-dependent hot-electron particle-in-cell solver.

This module only *describes* problems: layer stacks, per-channel material parameters,
interface transmission tables, the pump schedule and the bin edges.  It contains none of
the particle update (push, scattering, deposition).  The same `Problem` objects are handed
to the CPU oracle (`oracle/`) and to the device library, so both sides see bit-identical
inputs.

Physical model (Nenno, Rethfeld, Schneider, arXiv:1807.04733):
  * 1-D transport along z with speed v_sigma(E) and direction cos(theta) (Sec. II, Eq. 9);
  * effective lifetime 1/tau_eff = 1/tau_el + 1/tau_sigma(E) (Eq. 2);
  * inelastic events spawn secondaries with the equilibrium polarisation P0 (Eq. 19),
    which vanishes in the non-magnetic layer;
  * stochastic transmission at Fe/Au interfaces, full reflection at vacuum (Sec. III.A).
The numbers used here (velocities, tau0, transmissions) are the synthetic tables of the
standard workloads; the ab-initio curves of the paper's Fig. 1 are not available.

Conventions shared by both implementations (these are *input formats*, not arithmetic):
  * energies are uint32 fixed point above E_F with an LSB of 2^-30 eV;
  * interfaces lie on multiples of 2^-6 nm so they are exact in binary32;
  * channel c = (material, spin local to the layer); `ch_of[l, s]` maps layer l and global
    spin s (0 = up = emitter majority, 1 = down) to a channel;
  * `tt_of[k, d, s]` maps interface k (between layers k and k+1), direction d (0: +z,
    1: -z) and global spin s to a transmission table `T[t, :]`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

E_LSB_BITS = 30
E_ONE = 1 << E_LSB_BITS          # 1 eV in fixed point
Z_GRID = 1.0 / 64.0              # interface grid (nm)

# channel pool (index into v / inv_tau0)
FE_MAJ, FE_MIN, AU_UP, AU_DN = 0, 1, 2, 3
CHANNEL_NAMES = ("Fe_maj", "Fe_min", "Au_up", "Au_dn")
# transmission-table pool
T_FEAU_MAJ, T_FEAU_MIN, T_AUFE_MAJ, T_AUFE_MIN, T_ONE = 0, 1, 2, 3, 4

# synthetic material tables of the standard workloads (nm/fs, fs)
V_FE_MAJ, V_FE_MIN, V_AU = 0.6, 0.3, 1.0
TAU0_FE_MAJ, TAU0_FE_MIN, TAU0_AU = 20.0, 8.0, 40.0
T_FEAU_UP, T_FEAU_DN = 0.8, 0.4
P0_FE = 0.2                      # equilibrium polarisation of Fe (60/40 split)
SPIN_UP_FRAC = 0.6


def e_fx(ev: float) -> int:
    """Energy in eV -> uint32 fixed point (LSB 2^-30 eV)."""
    v = int(round(ev * E_ONE))
    if not (0 <= v < (1 << 32)):
        raise ValueError(f"energy {ev} eV outside the fixed-point range")
    return v


def snap_z(z: float) -> float:
    """Round a layer thickness / position to the 2^-6 nm interface grid."""
    return round(z / Z_GRID) * Z_GRID


@dataclass
class Layer:
    material: str            # "Fe" or "Au"
    thickness: float         # nm
    magnet: int = 0          # +1 / -1 for Fe (emitter = +1), 0 for Au


@dataclass
class Instance:
    """One layer stack with its parameters, pump and depth binning."""
    z_bound: np.ndarray      # (L+1,) f64, nm
    ch_of: np.ndarray        # (L, 2) i32
    v: np.ndarray            # (C,) f64, nm/fs
    inv_tau0: np.ndarray     # (C,) f64, 1/fs   (tau = tau0 * (1 eV / E)^tau_exp)
    inv_tau_el: np.ndarray   # (L,) f64, 1/fs   (0 = no elastic channel)
    P0: np.ndarray           # (L,) f64, equilibrium polarisation for secondaries
    T: np.ndarray            # (NT, TE) f64, transmission tables
    tt_of: np.ndarray        # (L-1, 2, 2) i32
    T_scale: float           # (TE-1) / E_max_table  [1/eV]; unused when TE == 1
    src_z_lo: float
    src_z_hi: float
    src_lambda: float        # exponential depth scale (nm); 0 = uniform in [lo, hi)
    src_cd: float            # 1 - exp(-(hi-lo)/lambda), precomputed input
    src_up_frac: float
    src_e_lo: np.ndarray     # (2,) u32: E0 = e_lo[s] + floor(w * e_span[s] / 2^32)
    src_e_span: np.ndarray   # (2,) u32
    sched: np.ndarray        # (n_steps,) i64: primaries injected at the start of step n
    root_offset: int         # global root id of this instance's first primary
    nz: int                  # depth bins
    inv_dz: float            # 1 / depth-bin width (1/nm)
    layers: List[Layer] = field(default_factory=list)
    # optional energy-dependent channels: speed v_tab[c, k] and relative inelastic rate
    # r_tab[c, k] (1/tau = inv_tau0[c] * r) at E = k / e_scale eV; None = constant speed
    # and tau = tau0 (1 eV/E)^tau_exp
    v_tab: Optional[np.ndarray] = None
    r_tab: Optional[np.ndarray] = None
    e_scale: float = 0.0
    # optional superparticle weights (Eq. 10): a primary of spin s and initial energy E0
    # carries the weight interpolated from w_tab[s, k] at E = k / w_scale eV (clamped);
    # None = weight 1.  Used when Problem.weighted is set.
    w_tab: Optional[np.ndarray] = None
    w_scale: float = 0.0

    @property
    def e_nodes(self) -> int:
        return 0 if self.v_tab is None else int(self.v_tab.shape[1])

    @property
    def n_layers(self) -> int:
        return len(self.z_bound) - 1

    @property
    def n_primaries(self) -> int:
        return int(self.sched.sum())

    @property
    def n_channels(self) -> int:
        return len(self.v)

    @property
    def n_ttables(self) -> int:
        return self.T.shape[0]

    @property
    def t_entries(self) -> int:
        return self.T.shape[1]


@dataclass
class Problem:
    instances: List[Instance]
    seed: int
    dt: float
    n_steps: int
    tau_exp: int = 2
    e_min_fx: int = e_fx(0.1)
    secondaries: bool = True
    state_fp64: bool = False
    e_edges: np.ndarray = field(default_factory=lambda: np.array([0], np.uint32))
    dens_stride: int = 1
    cur_stride: int = 1
    name: str = ""
    gen_moment: bool = False      # also bin the generation label (with the density)
    absorb_next: bool = False     # below E_min: removed at the next event, not at once
    weighted: bool = False        # moments are weighted sums (Eq. 10)

    @property
    def n_ebins(self) -> int:
        return len(self.e_edges)

    @property
    def n_dslots(self) -> int:
        return (self.n_steps + self.dens_stride - 1) // self.dens_stride

    @property
    def n_cslots(self) -> int:
        return (self.n_steps + self.cur_stride - 1) // self.cur_stride

    def dens_shape(self, i: int):
        return (self.n_dslots, self.instances[i].nz, self.n_ebins, 2)

    def cur_shape(self, i: int):
        return (self.n_cslots, self.instances[i].nz, 2)

    def gen_shape(self, i: int):
        return (self.n_dslots, self.instances[i].nz, 2)

    @property
    def n_primaries(self) -> int:
        return sum(inst.n_primaries for inst in self.instances)


# ----------------------------------------------------------------------------- builders

def energy_edges(width_ev: float, e_max_ev: float) -> np.ndarray:
    """Lower edges of uniform energy bins [k*w, (k+1)*w), k < e_max/w (fixed point)."""
    n = int(round(e_max_ev / width_ev))
    return np.array([e_fx(k * width_ev) for k in range(n)], dtype=np.uint32)


def gaussian_schedule(n_primaries: int, fwhm: float, t0: float, dt: float,
                      n_steps: int) -> np.ndarray:
    """Primaries injected at the start of each step for a Gaussian pump.

    Step n collects the pump between t_n - dt/2 and t_n + dt/2, i.e. the second half of
    the previous step's Source(dt/2) and the first half of this step's (Strang splitting,
    Eq. 15).  Counts are differences of the rounded cumulative pump, so they sum to
    `n_primaries` exactly once the pulse is over.
    """
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))

    def cum(t):
        return n_primaries * 0.5 * (1.0 + math.erf((t - t0) / (sigma * math.sqrt(2.0))))

    sched = np.zeros(n_steps, np.int64)
    prev = 0
    for n in range(n_steps):
        hi = int(round(cum(n * dt + 0.5 * dt)))
        if n == n_steps - 1:
            hi = n_primaries
        sched[n] = hi - prev
        prev = hi
    return sched


def instant_schedule(n_primaries: int, n_steps: int) -> np.ndarray:
    s = np.zeros(n_steps, np.int64)
    s[0] = n_primaries
    return s


def make_instance(layers: Sequence[Layer], *, n_primaries: int, n_steps: int,
                  e0_ev=(1.5, 1.5), e_span_ev=(0.0, 0.0),
                  src_layer: int = 0, src_lambda: float = 15.0,
                  up_frac: float = SPIN_UP_FRAC,
                  sched: Optional[np.ndarray] = None, root_offset: int = 0,
                  dz: float = 1.0, transparent: bool = False,
                  tau_el: float = 0.0, tau0_scale=(1.0, 1.0, 1.0, 1.0),
                  T_values=None, T_tables: Optional[np.ndarray] = None,
                  T_emax: float = 2.0, p0_fe: float = P0_FE,
                  v=(V_FE_MAJ, V_FE_MIN, V_AU, V_AU),
                  tau0=(TAU0_FE_MAJ, TAU0_FE_MIN, TAU0_AU, TAU0_AU)) -> Instance:
    """Build an `Instance` from a layer list.

    T_values: (FeAu_maj, FeAu_min, AuFe_maj, AuFe_min) scalars; default the standard
    table with the same value in both directions, keyed by the spin local to the Fe
    layer the interface touches.  T_tables: (4, TE) tables on [0, T_emax] eV instead.
    """
    L = len(layers)
    z = [0.0]
    for ly in layers:
        z.append(snap_z(z[-1] + ly.thickness))
    z_bound = np.array(z, np.float64)
    if np.any(np.diff(z_bound) <= 0):
        raise ValueError("layer thicknesses must be positive on the 2^-6 nm grid")

    ch_of = np.zeros((L, 2), np.int32)
    P0 = np.zeros(L, np.float64)
    for l, ly in enumerate(layers):
        if ly.material == "Fe":
            if ly.magnet not in (1, -1):
                raise ValueError("Fe layers need magnet = +1 or -1")
            ch_of[l, 0] = FE_MAJ if ly.magnet > 0 else FE_MIN
            ch_of[l, 1] = FE_MIN if ly.magnet > 0 else FE_MAJ
            P0[l] = p0_fe * ly.magnet
        elif ly.material == "Au":
            ch_of[l] = (AU_UP, AU_DN)
        else:
            raise ValueError(f"unknown material {ly.material}")

    if T_tables is not None:
        tabs = np.asarray(T_tables, np.float64)
        if tabs.shape[0] != 4:
            raise ValueError("T_tables must hold 4 tables")
        TE = tabs.shape[1]
        T_scale = (TE - 1) / T_emax
    else:
        if T_values is None:
            T_values = (T_FEAU_UP, T_FEAU_DN, T_FEAU_UP, T_FEAU_DN)
        tabs = np.array(T_values, np.float64).reshape(4, 1)
        TE = 1
        T_scale = 0.0
    if transparent:
        tabs = np.ones_like(tabs)
    need_one = any(layers[k].material == layers[k + 1].material for k in range(L - 1))
    T = np.concatenate([tabs, np.ones((1, TE))]) if need_one else tabs

    tt_of = np.zeros((max(L - 1, 0), 2, 2), np.int32)
    for k in range(L - 1):
        a, b = layers[k], layers[k + 1]
        for s in range(2):
            if a.material == b.material:
                tt_of[k, :, s] = T_ONE
                continue
            fe = a if a.material == "Fe" else b
            local_maj = (s == 0) == (fe.magnet > 0)
            feau = T_FEAU_MAJ if local_maj else T_FEAU_MIN
            aufe = T_AUFE_MAJ if local_maj else T_AUFE_MIN
            # direction 0 is +z (from layer k to k+1)
            tt_of[k, 0, s] = feau if a.material == "Fe" else aufe
            tt_of[k, 1, s] = aufe if a.material == "Fe" else feau

    inv_tau0 = np.array([1.0 / (t * sc) for t, sc in zip(tau0, tau0_scale)], np.float64)
    inv_tau_el = np.full(L, (1.0 / tau_el) if tau_el > 0 else 0.0, np.float64)

    src_lo = float(z_bound[src_layer])
    src_hi = float(z_bound[src_layer + 1])
    cd = -math.expm1(-(src_hi - src_lo) / src_lambda) if src_lambda > 0 else 0.0
    if sched is None:
        sched = instant_schedule(n_primaries, n_steps)
    sched = np.asarray(sched, np.int64)
    if int(sched.sum()) != n_primaries or len(sched) != n_steps:
        raise ValueError("schedule must cover n_steps and sum to n_primaries")
    e_lo = np.array([e_fx(e0_ev[0]), e_fx(e0_ev[1])], np.uint32)
    e_span = np.array([e_fx(e_span_ev[0]), e_fx(e_span_ev[1])], np.uint32)
    nz = int(math.ceil(z_bound[-1] / dz - 1e-9))
    return Instance(z_bound=z_bound, ch_of=ch_of, v=np.array(v, np.float64),
                    inv_tau0=inv_tau0, inv_tau_el=inv_tau_el, P0=P0, T=T, tt_of=tt_of,
                    T_scale=float(T_scale), src_z_lo=src_lo, src_z_hi=src_hi,
                    src_lambda=float(src_lambda), src_cd=float(cd),
                    src_up_frac=float(up_frac), src_e_lo=e_lo, src_e_span=e_span,
                    sched=sched, root_offset=int(root_offset), nz=nz, inv_dz=1.0 / dz,
                    layers=list(layers))


def bilayer(fe: float = 15.0, au: float = 100.0):
    return [Layer("Fe", fe, +1), Layer("Au", au, 0)]


def spin_valve(fe1: float = 15.0, au: float = 100.0, fe2: float = 15.0, parallel=True):
    return [Layer("Fe", fe1, +1), Layer("Au", au, 0), Layer("Fe", fe2, +1 if parallel else -1)]


def synthetic_channel_tables(v: Sequence[float], nodes: int = 64, e_max: float = 2.0):
    """Smooth synthetic energy dependences standing in for Fig. 1 (the ab-initio curves are
    not available): speeds rising as sqrt(1 + E / 1 eV) from the channel's speed at
    E = 0, and relative inelastic rates (E/1 eV)^2 + 0.05 (Fermi-liquid-like, finite at
    E_F).  Returns (v_tab (C, nodes), r_tab (C, nodes), e_scale)."""
    e = np.arange(nodes) * (e_max / (nodes - 1))
    v_tab = np.stack([vc * np.sqrt(1.0 + e) for vc in v]).astype(np.float64)
    r_tab = np.stack([e * e + 0.05 for _ in v]).astype(np.float64)
    return v_tab, r_tab, (nodes - 1) / e_max


def importance_weights(inst: Instance, q_up: float = 0.5, nodes: int = 16,
                       e_max: float = 2.0, slope: float = 1.0):
    """Source importance sampling (Eq. 10 weights): the spin is sampled with probability
    q_up instead of the instance's src_up_frac p, and the energy uniformly in the pump
    window while the physical spectrum is taken proportional to 1 + slope * E / 1 eV over
    that window.  The weight of a primary is the ratio of physical to sampling density:
    (p / q_up or (1 - p) / (1 - q_up)) * (1 + slope E) / mean(1 + slope E).  Returns
    (src_up_frac to sample with, w_tab (2, nodes), w_scale)."""
    p = inst.src_up_frac
    e = np.arange(nodes) * (e_max / (nodes - 1))
    rows = []
    for s, ws in ((0, p / q_up), (1, (1.0 - p) / (1.0 - q_up))):
        lo = inst.src_e_lo[s] * 2.0 ** -30
        hi = (int(inst.src_e_lo[s]) + int(inst.src_e_span[s])) * 2.0 ** -30
        rows.append(ws * (1.0 + slope * e) / (1.0 + slope * 0.5 * (lo + hi)))
    return q_up, np.stack(rows).astype(np.float64), (nodes - 1) / e_max


def variant(problem: Problem, *, tau_el: Optional[float] = None, transparent: bool = False,
            secondaries: Optional[bool] = None, absorb_next: Optional[bool] = None,
            gen_moment: Optional[bool] = None, energy_tables: bool = False,
            weights: bool = False) -> Problem:
    """A copy of `problem` with the physics switches of the paper's comparisons (Sec. V):
    an elastic channel of lifetime tau_el in every layer, transparent interfaces (T = 1),
    secondaries on / off, removal at the next event, the generation moment,
    energy-dependent speeds and lifetimes (synthetic tables), and weighted superparticles
    from importance sampling of the source (Eq. 10)."""
    insts = []
    for it in problem.instances:
        it = replace(it)
        if tau_el is not None:
            it.inv_tau_el = np.full(it.n_layers, 1.0 / tau_el if tau_el > 0 else 0.0)
        if transparent:
            it.T = np.ones_like(it.T)
        if energy_tables:
            it.v_tab, it.r_tab, it.e_scale = synthetic_channel_tables(it.v)
        if weights:
            it.src_up_frac, it.w_tab, it.w_scale = importance_weights(it)
        insts.append(it)
    out = replace(problem, instances=insts)
    if weights:
        out.weighted = True
    if secondaries is not None:
        out.secondaries = secondaries
    if absorb_next is not None:
        out.absorb_next = absorb_next
    if gen_moment is not None:
        out.gen_moment = gen_moment
    return out


def with_root_offsets(instances: List[Instance]) -> List[Instance]:
    off = 0
    out = []
    for inst in instances:
        out.append(replace(inst, root_offset=off))
        off += inst.n_primaries
    return out


# ----------------------------------------------------------------------------- standard workloads

def config0(n_primaries: int = 100_000, n_steps: int = 300, seed: int = 0) -> Problem:
    """Fe(15)/Au(100) bilayer, mono-energetic 1.5 eV pump at t=0, FP64 state."""
    inst = make_instance(bilayer(), n_primaries=n_primaries, n_steps=n_steps)
    return Problem([inst], seed=seed, dt=1.0, n_steps=n_steps, state_fp64=True,
                   name="fe15_au100_bilayer_fp64")


def config1(parallel: bool = True, n_primaries: int = 10_000_000, n_steps: int = 1000,
            seed: int = 0, dens_stride: int = 1) -> Problem:
    """Fe(15)/Au(100)/Fe(15) spin valve (P or AP), E0 ~ U(0.5, 2.0) eV, FP32 state."""
    inst = make_instance(spin_valve(parallel=parallel), n_primaries=n_primaries,
                         n_steps=n_steps, e0_ev=(0.5, 0.5), e_span_ev=(1.5, 1.5))
    return Problem([inst], seed=seed, dt=0.5, n_steps=n_steps,
                   e_edges=energy_edges(0.05, 2.0), dens_stride=dens_stride,
                   name=f"fe15_au100_fe15_{'P' if parallel else 'AP'}_fp32")


def config2(n_instances: int = 256, seed: int = 0, n_steps: int = 500,
            prim_lo: float = 1e4, prim_hi: float = 1e6, param_seed: int = 0) -> Problem:
    """Batch of Fe/Au/Fe stacks with randomised thicknesses, pumps and parameters."""
    rng = np.random.default_rng(param_seed)
    insts = []
    for _ in range(n_instances):
        fe1 = snap_z(rng.uniform(5.0, 20.0))
        au = snap_z(rng.uniform(20.0, 200.0))
        fe2 = snap_z(rng.uniform(5.0, 20.0))
        npr = int(round(math.exp(rng.uniform(math.log(prim_lo), math.log(prim_hi)))))
        e0 = rng.uniform(0.8, 2.0)
        par = bool(rng.uniform() < 0.5)
        tau_sc = rng.uniform(0.7, 1.3, size=4)
        t_sc = rng.uniform(0.7, 1.3, size=2)
        tvals = (min(1.0, T_FEAU_UP * t_sc[0]), min(1.0, T_FEAU_DN * t_sc[1]))
        insts.append(make_instance(
            spin_valve(fe1, au, fe2, parallel=par), n_primaries=npr, n_steps=n_steps,
            e0_ev=(e0, e0), src_lambda=15.0, tau0_scale=tuple(tau_sc),
            T_values=(tvals[0], tvals[1], tvals[0], tvals[1])))
    insts = with_root_offsets(insts)
    return Problem(insts, seed=seed, dt=1.0, n_steps=n_steps,
                   e_edges=energy_edges(0.1, 2.0), dens_stride=5, cur_stride=1,
                   name=f"batched_{n_instances}_fe_au_fe")


def config3(n_primaries: int = 100_000_000, n_steps: int = 400, seed: int = 0,
            tau0_scale=(1.0, 1.0, 1.0, 1.0), T_values=None) -> Problem:
    """Fe(15)/Au(80) bilayer for the adjoint: 8 parameters (4 tau0, 4 T)."""
    if T_values is None:
        T_values = (T_FEAU_UP, T_FEAU_DN, T_FEAU_UP, T_FEAU_DN)
    inst = make_instance(bilayer(15.0, 80.0), n_primaries=n_primaries, n_steps=n_steps,
                         e0_ev=(0.5, 0.5), e_span_ev=(1.5, 1.5), tau0_scale=tau0_scale,
                         T_values=T_values)
    return Problem([inst], seed=seed, dt=1.0, n_steps=n_steps,
                   e_edges=energy_edges(0.05, 2.0), name="fe15_au80_adjoint")


def synthetic_T_tables(entries: int = 64, e_max: float = 2.0) -> np.ndarray:
    """Smooth synthetic energy-dependent transmissions (majority / minority)."""
    e = np.arange(entries) * (e_max / (entries - 1))
    up = 0.8 - 0.2 * (1.0 - e / 2.0) ** 2
    dn = 0.4 + 0.1 * np.sin(np.pi * e / 2.0)
    return np.stack([up, dn, up, dn]).astype(np.float64)


def config4(n_instances: int = 64, primaries_per_instance: int = 3_125_000,
            n_steps: int = 2000, seed: int = 0) -> Problem:
    """[Fe(10)/Au(30)]x5 multilayers, Gaussian pump (50 fs FWHM at 100 fs), T(E) tables."""
    layers = []
    for _ in range(5):
        layers += [Layer("Fe", 10.0, +1), Layer("Au", 30.0, 0)]
    dt = 0.5
    sched = gaussian_schedule(primaries_per_instance, 50.0, 100.0, dt, n_steps)
    tabs = synthetic_T_tables()
    insts = [make_instance(layers, n_primaries=primaries_per_instance, n_steps=n_steps,
                           e0_ev=(1.5, 1.0), sched=sched, T_tables=tabs)
             for _ in range(n_instances)]
    insts = with_root_offsets(insts)
    return Problem(insts, seed=seed, dt=dt, n_steps=n_steps,
                   e_edges=energy_edges(0.1, 2.0), dens_stride=4, cur_stride=1,
                   name=f"batched_{n_instances}_fe10_au30_x5_gaussian")


def homogeneous(thickness: float = 100.0, n_primaries: int = 1000, n_steps: int = 50,
                split_at: Optional[float] = None, e0_ev: float = 1.5, tau0: float = 40.0,
                tau_el: float = 0.0, tau_exp: int = 2, dt: float = 1.0, seed: int = 0,
                secondaries: bool = True, e_min_ev: float = 0.1, state_fp64: bool = True,
                src_lambda: float = 0.0, src=(None, None), up_frac: float = 0.5,
                e_edges=None, dz: float = 1.0) -> Problem:
    """A single Au slab (optionally split into two identical layers joined by T = 1)."""
    if split_at is None:
        layers = [Layer("Au", thickness)]
    else:
        layers = [Layer("Au", split_at), Layer("Au", thickness - split_at)]
    inst = make_instance(layers, n_primaries=n_primaries, n_steps=n_steps,
                         e0_ev=(e0_ev, e0_ev), src_lambda=src_lambda, up_frac=up_frac,
                         tau_el=tau_el, tau0=(TAU0_FE_MAJ, TAU0_FE_MIN, tau0, tau0), dz=dz)
    lo, hi = src
    if lo is not None:
        inst.src_z_lo, inst.src_z_hi = float(lo), float(hi)
    elif split_at is not None:
        inst.src_z_lo, inst.src_z_hi = 0.0, float(inst.z_bound[-1])
    if e_edges is None:
        e_edges = np.array([0], np.uint32)
    return Problem([inst], seed=seed, dt=dt, n_steps=n_steps, tau_exp=tau_exp,
                   e_min_fx=e_fx(e_min_ev), secondaries=secondaries,
                   state_fp64=state_fp64, e_edges=np.asarray(e_edges, np.uint32),
                   name="homogeneous")


def root_step(inst: Instance) -> np.ndarray:
    """Injection step of every local root (roots are numbered in injection order)."""
    return np.repeat(np.arange(len(inst.sched)), inst.sched)
