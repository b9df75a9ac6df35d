"""Seeded synthetic workloads shaped like the paper's test cases.

This module only *describes* runs and draws their random initial states; it
holds none of the method's arithmetic (no push, shape, deposit, field
update or initial momentum split).  Both the HIP library binding and the
FP64 oracle consume the objects defined here, and nothing else is shared
between them.

Units are the normalised ones of the library: c = eps0 = e = m_e = 1 and
laser angular frequency 1, so the laser wavelength is 2 pi, densities are
in units of the critical density and E in units of m_e c omega / e (a plane
wave of normalised amplitude a0 has |E| = a0).

Workloads (the paper's cases as restated for this project):
  neutral_medium_1d   laser in a neutral bound-electron medium, Sec. 3.1
  bragg_2d            x-ray Bragg scattering from a rotated lattice, Sec. 3.2
  ionised_slab_3d     3D partially ionised slab with free electrons
  mixed_precision_3d  Bragg-geometry 3D slab, 4 ions per cell
  adjoint_slab        2D neutral slab crossed by a spline-envelope pulse (gradient runs)
  bound_slab_1d       medium behind a vacuum gap (Sec. 3.1 observables)
  wakefield_crystal_2d  relativistic pulse in a pre-ionised gold lattice (Sec. 3.2, Fig. 6)
  multishell_medium_1d  medium of ions with two bound clouds each (linear response)
  multishell_slab_3d    3D medium of two-cloud ions (throughput of the multi-shell kernel)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

PERIODIC, OPEN, LASER = 0, 1, 2
POINT, TWO_BODY, MULTI_SHELL = 0, 1, 2

# physical constants (CODATA 2018)
ME_C2_EV = 510998.95            # electron rest energy, eV
AMU_IN_ME = 1822.888486209      # atomic mass unit in electron masses
AU_MASS_AMU = 196.966570        # gold
R_E_M = 2.8179403262e-15        # classical electron radius, m
HC_EV_NM = 1239.84198           # h c in eV nm

TWO_PI = 2.0 * math.pi
BASE_SEED = 20220808


@dataclass
class Laser:
    """Laser entering through x-min: E_inc = a0 sin^2(pi t'/t_env) sin(omega t' + phase),
    t' = t - t_delay - x, times exp(-r_perp^2 / waist^2) when waist > 0.  A non-empty
    `env` replaces sin^2 by sum_k env[k] N3(t'/h - k), h = t_env / (len(env) + 3),
    N3 the cardinal cubic B-spline on [0, 4]."""
    a0: float = 0.0
    omega: float = 1.0
    t_env: float = 0.0
    waist: float = 0.0
    yc: float = 0.0
    zc: float = 0.0
    phase: float = 0.0
    t_delay: float = 0.0
    pol: int = 1  # 1: E along y (in the x-y plane), 2: E along z
    angle: float = 0.0  # direction of travel from +x toward +y (plane waves only)
    env: Tuple[float, ...] = ()  # spline envelope coefficients (at most 64)


@dataclass
class Grid:
    ndim: int
    n: Tuple[int, int, int]
    dx: Tuple[float, float, float]
    dt: float
    bc_lo: Tuple[int, int, int] = (PERIODIC, PERIODIC, PERIODIC)
    bc_hi: Tuple[int, int, int] = (PERIODIC, PERIODIC, PERIODIC)
    pad: int = 3
    laser: Laser = field(default_factory=Laser)
    re_norm: float = 0.0  # 2 pi r_e / lambda_laser, for a_c = 0 species

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n[: self.ndim]))


@dataclass
class Species:
    """Real-particle charges/masses (units e, m_e).  A point species uses q1, m1.
    a_c: softening length; 0 derives it from omega_c and the grid's re_norm;
    math.inf selects the exact harmonic bond."""
    kind: int
    q1: float
    m1: float
    q2: float = 0.0
    m2: float = 0.0
    weight: float = 1.0
    omega_c: float = 0.0
    a_c: float = 0.0
    nu: float = 0.0
    nu_per_omega: float = 0.0
    name: str = ""
    # MULTI_SHELL: the nucleus is (q1, m1); each shell is a bound cloud
    # (charge, mass, omega_c, a_c) with its own bond to the nucleus
    shells: Tuple[Tuple[float, float, float, float], ...] = ()


@dataclass
class Particles:
    x: np.ndarray                       # (n, ndim) positions, centre of mass for two-body
    u1: np.ndarray                      # (n, 3) momentum per mass (centre of mass if u2 is None)
    delta: Optional[np.ndarray] = None  # (n, 3) r1 - r2; multi-shell (n, 3 K) r0 - r_k
    u2: Optional[np.ndarray] = None     # (n, 3); multi-shell (n, 3 K) the clouds
    omega_c: Optional[np.ndarray] = None
    weight: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Workload:
    name: str
    grid: Grid
    species: List[Tuple[Species, Particles]]
    steps: int
    precision: int = 64
    probes: List[Tuple[int, Tuple[int, int, int]]] = field(default_factory=list)
    notes: str = ""

    @property
    def n_particles(self) -> int:
        return sum(p.n for _, p in self.species)


def rng_for(case_id: int, stream: int = 0) -> np.random.Generator:
    """Counter-based Philox stream keyed by (seed + case id, stream)."""
    return np.random.Generator(np.random.Philox(key=[BASE_SEED + case_id, stream]))


def gold_ion(z_bound: int, q_c: float):
    """Two-body gold macro-ion charges/masses: q2 = -Z_b, m2 = Z_b, q1 = q_c - q2, m1 = m_c - m2."""
    m_c = AU_MASS_AMU * AMU_IN_ME
    q2, m2 = -float(z_bound), float(z_bound)
    return q_c - q2, m_c - m2, q2, m2


def bound_plasma_density(q1, m1, q2, m2, omega_pb):
    """Ion density for which the bound-oscillator plasma frequency
    omega_pb^2 = n q_r^2 / m_r takes the requested value (workload recipe)."""
    mc = m1 + m2
    m_r = m1 * m2 / mc
    q_r = (q1 * m2 - q2 * m1) / mc
    return omega_pb ** 2 * m_r / q_r ** 2


def thermal_sigma(t_ev: float, mass_me: float) -> float:
    """Standard deviation of u = p/(m c) per component for temperature t_ev."""
    return math.sqrt(t_ev / (mass_me * ME_C2_EV))


def stratified_positions(rng, lo, hi, ppc, dx, ndim):
    """ppc particles per cell over cells lo..hi-1 (per dimension), cells
    enumerated x fastest; each particle uniform within its own sub-stratum
    along x (ppc slices) and uniform along the other dimensions."""
    counts = [int(hi[d] - lo[d]) for d in range(ndim)]
    ncell = int(np.prod(counts))
    n = ncell * ppc
    x = np.empty((n, ndim), dtype=np.float64)
    # particle p lives in cell p // ppc, sub-stratum p % ppc
    cidx = np.arange(n, dtype=np.int64) // ppc
    sub = (np.arange(n, dtype=np.int64) % ppc).astype(np.float64)
    rem = cidx
    for d in range(ndim):
        cd = (rem % counts[d]).astype(np.float64) + lo[d]
        rem = rem // counts[d]
        if d == 0:
            x[:, 0] = (cd + (sub + rng.random(n)) / ppc) * dx[0]
        else:
            x[:, d] = (cd + rng.random(n)) * dx[d]
    return x


def _probe_list(ndim, comp, cells):
    out = []
    for c in cells:
        idx = [0, 0, 0]
        for d in range(ndim):
            idx[d] = int(c[d]) if isinstance(c, (tuple, list)) else (int(c) if d == 0 else 0)
        out.append((comp, tuple(idx)))
    return out


# --------------------------------------------------------------------------
# Case 1: laser in a neutral bound-electron medium (Sec. 3.1), 1D, FP64
# --------------------------------------------------------------------------

def neutral_medium_1d(cells: int = 2048, ppc: int = 8, steps: int = 1000,
                      omega_c: float = 3.0, omega_pb: float = 0.9, a0: float = 1e-3,
                      t_ev: float = 1.0, cycles: int = 10, a_c: float = 0.0,
                      probes=(32, 224), case_id: int = 1) -> Workload:
    dx = TWO_PI / 64.0
    dt = 0.98 * dx
    lam_m = 12.4e-9  # 0.1 keV photons, as in Sec. 3.1
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, pol=1)
    grid = Grid(1, (cells, 1, 1), (dx, 1.0, 1.0), dt, (LASER, PERIODIC, PERIODIC),
                (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                re_norm=TWO_PI * R_E_M / lam_m)
    q1, m1, q2, m2 = gold_ion(78, 0.0)
    n_ion = bound_plasma_density(q1, m1, q2, m2, omega_pb)
    w = n_ion * dx / ppc
    sp = Species(TWO_BODY, q1, m1, q2, m2, weight=w, omega_c=omega_c, a_c=a_c, name="Au_Zb78")
    rng = rng_for(case_id)
    pad = grid.pad
    x = stratified_positions(rng, [pad], [cells - pad], ppc, grid.dx, 1)
    n = x.shape[0]
    sig = thermal_sigma(t_ev, m1 + m2)
    uc = rng.normal(0.0, sig, size=(n, 3))
    parts = Particles(x=x, u1=uc)
    return Workload("neutral_medium_1d", grid, [(sp, parts)], steps, 64,
                    probes=_probe_list(1, 1, list(probes)),
                    notes=f"{n} two-body ions, omega_c={omega_c}, omega_pb={omega_pb}")


def ionised_medium_1d(cells: int = 2048, ppc: int = 8, steps: int = 1000,
                      omega_pb: float = 0.9, a0: float = 1e-4, cycles: int = 10,
                      wc_range=(1.5, 4.0), nu_per_omega: float = 0.01,
                      probes=(32, 224), case_id: int = 13) -> Workload:
    """1D counterpart of the ionised slab for its linear-response check:
    cold gold ions with one free electron each (q_c = +1), every ion with
    its own omega_c drawn uniformly from wc_range (softening length derived
    from it), friction nu_per_omega * omega_c, free electrons at the ions'
    density, plane wave polarised along y entering at x-min."""
    dx = TWO_PI / 64.0
    dt = 0.98 * dx
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, pol=1)
    grid = Grid(1, (cells, 1, 1), (dx, 1.0, 1.0), dt, (LASER, PERIODIC, PERIODIC),
                (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                re_norm=TWO_PI * R_E_M / 12.4e-9)
    q1, m1, q2, m2 = gold_ion(78, 1.0)
    n_ion = bound_plasma_density(q1, m1, q2, m2, omega_pb)
    w = n_ion * dx / ppc
    ion = Species(TWO_BODY, q1, m1, q2, m2, weight=w, omega_c=0.5 * sum(wc_range), a_c=0.0,
                  nu_per_omega=nu_per_omega, name="Au_q1_cold")
    pad = grid.pad
    rng_i = rng_for(case_id, 0)
    xi = stratified_positions(rng_i, [pad], [cells - pad], ppc, grid.dx, 1)
    ni = xi.shape[0]
    wci = rng_i.uniform(wc_range[0], wc_range[1], size=ni)
    rng_e = rng_for(case_id, 1)
    xe = stratified_positions(rng_e, [pad], [cells - pad], ppc, grid.dx, 1)
    ele = Species(POINT, -1.0, 1.0, weight=w, name="e_cold")
    species = [(ion, Particles(x=xi, u1=np.zeros((ni, 3)), omega_c=wci)),
               (ele, Particles(x=xe, u1=np.zeros((xe.shape[0], 3))))]
    return Workload("ionised_medium_1d", grid, species, steps, 64,
                    probes=_probe_list(1, 1, list(probes)),
                    notes=f"{ni} cold two-body ions with omega_c in {wc_range} + {ni} electrons")


def multishell_medium_1d(cells: int = 2048, ppc: int = 8, steps: int = 1000,
                         nucleus=(8.0, 20.0), shells=((-5.0, 5.0, 1.6, math.inf),
                                                      (-3.0, 3.0, 2.4, math.inf)),
                         density: float = 0.01, nu: float = 0.02, a0: float = 1e-4,
                         cycles: int = 10, probes=(32, 224), case_id: int = 14) -> Workload:
    """1D medium of neutral multi-shell ions (a nucleus and two clouds with
    their own bonds) for the linear-response check of the multi-resonance
    permittivity: ions at rest, `density` ions per (c/omega)^3 (units of
    n_c), friction nu on each nucleus-cloud pair, weak plane wave polarised
    along y entering at x-min, E_y probes at two cells."""
    dx = TWO_PI / 64.0
    dt = 0.98 * dx
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, pol=1)
    grid = Grid(1, (cells, 1, 1), (dx, 1.0, 1.0), dt, (LASER, PERIODIC, PERIODIC),
                (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser, re_norm=1e-3)
    w = density * dx / ppc
    sp = Species(MULTI_SHELL, nucleus[0], nucleus[1], weight=w, nu=nu, shells=tuple(shells),
                 name="two_shell")
    pad = grid.pad
    x = stratified_positions(rng_for(case_id, 0), [pad], [cells - pad], ppc, grid.dx, 1)
    n = x.shape[0]
    K = len(shells)
    parts = Particles(x=x, u1=np.zeros((n, 3)), delta=np.zeros((n, 3 * K)),
                      u2=np.zeros((n, 3 * K)))
    return Workload("multishell_medium_1d", grid, [(sp, parts)], steps, 64,
                    probes=_probe_list(1, 1, list(probes)),
                    notes=f"{n} neutral two-shell ions at rest")


def multishell_slab_3d(n=(256, 128, 128), ppc: int = 2, steps: int = 60,
                       nucleus=(26.0, 55.845 * 1822.888), shells=((-8.0, 8.0, 3.0, 0.0),
                                                                 (-18.0, 18.0, 1.2, 0.0)),
                       density: float = 0.01, nu: float = 0.01, a0: float = 1e-3,
                       waist_lambda: float = 8.0, cycles: int = 10, precision: int = 32,
                       case_id: int = 15) -> Workload:
    """Medium of neutral multi-shell ions filling the box between the
    particle walls (the throughput case of the multi-shell kernel): an
    iron-like nucleus with two bound clouds (8 and 18 electrons, restoring
    frequencies 3 and 1.2, softening lengths derived from them), `ppc` ions
    per cell at rest, `density` ions per (c/omega)^3, friction nu on each
    nucleus-cloud pair; Gaussian laser a0 through x-min, periodic y and z."""
    dx = TWO_PI / 24.0
    dt = 0.98 * dx / math.sqrt(3.0)
    lam_m = 12.4e-9
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, waist=waist_lambda * TWO_PI,
                  yc=0.5 * n[1] * dx, zc=0.5 * n[2] * dx, pol=1)
    grid = Grid(3, tuple(n), (dx, dx, dx), dt, (LASER, PERIODIC, PERIODIC),
                (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                re_norm=TWO_PI * R_E_M / lam_m)
    w = density * dx ** 3 / ppc
    sp = Species(MULTI_SHELL, nucleus[0], nucleus[1], weight=w, nu=nu, shells=tuple(shells),
                 name="two_shell_3d")
    rng = rng_for(case_id, 0)
    x = stratified_positions(rng, [grid.pad, 0, 0], [n[0] - grid.pad, n[1], n[2]], ppc,
                             grid.dx, 3)
    m = x.shape[0]
    K = len(shells)
    parts = Particles(x=x, u1=np.zeros((m, 3)), delta=np.zeros((m, 3 * K)),
                      u2=np.zeros((m, 3 * K)))
    return Workload("multishell_slab_3d", grid, [(sp, parts)], steps, precision,
                    notes=f"{m} neutral two-shell ions at rest")


def bound_slab_1d(cells: int = 1536, x_cells=(256, 1536), ppc: int = 4, steps: int = 2200,
                  omega_c: float = 3.0, omega_pb: float = 0.9, a0: float = 1e-4,
                  cycles: int = 10, dx_per_lambda: int = 64, case_id: int = 11) -> Workload:
    """Neutral bound-electron medium filling x_cells (cells) after a vacuum
    gap, for the observables of Sec. 3.1 (group velocity, reflection phase):
    cold two-body gold ions (delta = 0, at rest), plane wave polarised along
    y entering at x-min.  The medium's far end is the particle wall
    (x_cells[1] may reach cells - pad)."""
    dx = TWO_PI / float(dx_per_lambda)
    dt = 0.98 * dx
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, pol=1)
    grid = Grid(1, (cells, 1, 1), (dx, 1.0, 1.0), dt, (LASER, PERIODIC, PERIODIC),
                (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                re_norm=TWO_PI * R_E_M / 12.4e-9)
    q1, m1, q2, m2 = gold_ion(78, 0.0)
    n_ion = bound_plasma_density(q1, m1, q2, m2, omega_pb)
    sp = Species(TWO_BODY, q1, m1, q2, m2, weight=n_ion * dx / ppc, omega_c=omega_c,
                 a_c=math.inf, name="Au_Zb78_cold")
    lo, hi = x_cells[0], min(x_cells[1], cells - grid.pad)
    x = stratified_positions(rng_for(case_id), [lo], [hi], ppc, grid.dx, 1)
    parts = Particles(x=x, u1=np.zeros((x.shape[0], 3)))
    return Workload("bound_slab_1d", grid, [(sp, parts)], steps, 64,
                    notes=f"medium cells {lo}..{hi}, omega_c={omega_c}, omega_pb={omega_pb}")


def adjoint_slab(ndim: int = 2, cells=(2048, 1024), slab=(64, 448), probe_x: int = 512,
                 ppc: int = 16, steps: int = 1024, omega_c: float = 3.0, omega_pb: float = 0.9,
                 nu: float = 0.03, a_c: float = math.inf, n_env: int = 64, cycles: float = 4.0,
                 a0: float = 1e-4, waist_frac: float = 0.3, dx_per_lambda: int = 32,
                 case_id: int = 5) -> Workload:
    """Gradient-run case: a neutral bound-electron slab (cold two-body gold
    ions, Z_b = 78, ppc per cell over x cells slab[0]..slab[1] and every y,
    z) crossed by a pulse from x-min whose temporal envelope is a cubic
    B-spline series of n_env coefficients over `cycles` laser periods
    (initial coefficients: sin^2 sampled at the basis centres); y (and z)
    periodic, a wide Gaussian profile (waist = waist_frac * L_y; plane wave
    in 1D).  Probes on the plane x = probe_x behind the slab: E_y at
    (probe_x, j, k), then B_z at (probe_x - 1, j, k), then B_z at
    (probe_x, j, k), each over every (j, k) with j fastest (the transmitted
    Poynting flux and phase)."""
    dx = TWO_PI / float(dx_per_lambda)
    dt = 0.98 * dx / math.sqrt(float(ndim))
    nx = int(cells[0])
    ny = int(cells[1]) if ndim > 1 else 1
    nz = int(cells[2]) if ndim > 2 else 1
    t_env = cycles * TWO_PI
    h = t_env / (n_env + 3)
    env = tuple(math.sin(math.pi * (k + 2) * h / t_env) ** 2 for k in range(n_env))
    Ly = ny * dx
    laser = Laser(a0=a0, omega=1.0, t_env=t_env, pol=1, env=env,
                  waist=waist_frac * Ly if ndim > 1 else 0.0, yc=0.5 * Ly if ndim > 1 else 0.0,
                  zc=0.5 * nz * dx if ndim > 2 else 0.0)
    if ndim == 3:
        grid = Grid(3, (nx, ny, nz), (dx, dx, dx), dt, (LASER, PERIODIC, PERIODIC),
                    (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                    re_norm=TWO_PI * R_E_M / 12.4e-9)
    elif ndim == 1:
        grid = Grid(1, (nx, 1, 1), (dx, 1.0, 1.0), dt, (LASER, PERIODIC, PERIODIC),
                    (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                    re_norm=TWO_PI * R_E_M / 12.4e-9)
    else:
        grid = Grid(2, (nx, ny, 1), (dx, dx, 1.0), dt, (LASER, PERIODIC, PERIODIC),
                    (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                    re_norm=TWO_PI * R_E_M / 12.4e-9)
    q1, m1, q2, m2 = gold_ion(78, 0.0)
    n_ion = bound_plasma_density(q1, m1, q2, m2, omega_pb)
    cell_vol = dx ** ndim
    sp = Species(TWO_BODY, q1, m1, q2, m2, weight=n_ion * cell_vol / ppc, omega_c=omega_c,
                 a_c=a_c, nu=nu, name="Au_Zb78_cold")
    lo = [slab[0]] + [0] * (ndim - 1)
    hi = [min(slab[1], nx - grid.pad)] + [ny, nz][:ndim - 1]
    x = stratified_positions(rng_for(case_id), lo, hi, ppc, grid.dx, ndim)
    parts = Particles(x=x, u1=np.zeros((x.shape[0], 3)))
    plane = [(j, k) for k in range(nz) for j in range(ny)]
    probes = ([(1, (probe_x, j, k)) for j, k in plane] +
              [(5, (probe_x - 1, j, k)) for j, k in plane] +
              [(5, (probe_x, j, k)) for j, k in plane])
    return Workload("adjoint_slab", grid, [(sp, parts)], steps, 64, probes=probes,
                    notes=f"slab {slab}, probe plane x={probe_x}, omega_c={omega_c}, nu={nu}")


# --------------------------------------------------------------------------
# Case 2: Bragg scattering from a rotated square lattice (Sec. 3.2), 2D
# --------------------------------------------------------------------------

def bragg_2d(cells: int = 4096, slab: int = 1024, steps: int = 4000, d_over_lambda: float = 1.5,
             omega_c: float = 0.5, a0: float = 1e-4, cycles: int = 20,
             waist_lambda: float = 12.0, jitter: float = 0.01, precision: int = 64,
             weight_scale: float = 1.0, case_id: int = 2) -> Workload:
    dx = TWO_PI / 32.0
    dt = 0.98 * dx / math.sqrt(2.0)
    lam = TWO_PI
    d = d_over_lambda * lam
    # gold lattice constant d = n^{-1/3} = 0.2569 nm fixes the laser wavelength
    d_m = (5.9e28) ** (-1.0 / 3.0)
    lam_m = d_m / d_over_lambda
    re_norm = TWO_PI * R_E_M / lam_m
    theta_b = math.asin(lam / (2.0 * d))
    Ly = cells * dx
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, waist=waist_lambda * lam,
                  yc=0.5 * Ly, pol=1)
    grid = Grid(2, (cells, cells, 1), (dx, dx, 1.0), dt, (LASER, OPEN, PERIODIC),
                (OPEN, OPEN, PERIODIC), pad=3, laser=laser, re_norm=re_norm)
    q1, m1, q2, m2 = gold_ion(78, 0.0)
    # one site = one column of atoms along z with spacing d: 1/d atoms per unit
    # length, i.e. 4 pi re_norm / d in units of n_c (c/omega)^2
    w = weight_scale * 4.0 * math.pi * re_norm / d
    sp = Species(TWO_BODY, q1, m1, q2, m2, weight=w, omega_c=omega_c, a_c=0.0, name="Au_lattice")
    rng = rng_for(case_id)
    c0 = 0.5 * cells * dx
    half = 0.5 * slab * dx
    m = int(math.ceil(2.0 * half * math.sqrt(2.0) / d)) + 2
    ii, jj = np.meshgrid(np.arange(-m, m + 1), np.arange(-m, m + 1), indexing="ij")
    a = ii.ravel() * d
    b = jj.ravel() * d
    ct, st = math.cos(theta_b), math.sin(theta_b)
    xs = c0 + a * ct - b * st
    ys = c0 + a * st + b * ct
    keep = (np.abs(xs - c0) < half) & (np.abs(ys - c0) < half)
    xs, ys = xs[keep], ys[keep]
    n = xs.size
    xs = xs + rng.normal(0.0, jitter * d, n)
    ys = ys + rng.normal(0.0, jitter * d, n)
    x = np.stack([xs, ys], axis=1)
    parts = Particles(x=x, u1=np.zeros((n, 3)))
    return Workload("bragg_2d", grid, [(sp, parts)], steps, precision,
                    notes=f"{n} lattice sites, d={d_over_lambda} lambda, theta_B={theta_b:.6f}")


def wakefield_crystal_2d(cells=(4096, 4096), slab=(2048, 1024), steps: int = 4000,
                         d_over_lambda: float = 1.5, omega_c: float = 0.5, a0: float = 3.0,
                         cycles: int = 20, waist_lambda: float = 12.0, free_per_ion: int = 30,
                         z_bound_neutral: int = 78, ppc_e: int = 1, t_e_ev: float = 10.0,
                         jitter: float = 0.01, precision: int = 64,
                         case_id: int = 6) -> Workload:
    """The Bragg lattice of bragg_2d, longer along x, pre-ionised with
    `free_per_ion` free electrons per ion, driven by a relativistic pulse
    (a0 = 3): Sec. 3.2, the wakefield paragraph.  Each site's ion keeps
    z_bound_neutral - free_per_ion bound electrons (net charge
    +free_per_ion); the free electrons fill the crystal region uniformly
    (ppc_e per cell, stratified, thermal at t_e_ev) with the weight that
    makes the region neutral."""
    nx, ny = cells
    dx = TWO_PI / 32.0
    dt = 0.98 * dx / math.sqrt(2.0)
    lam = TWO_PI
    d = d_over_lambda * lam
    d_m = (5.9e28) ** (-1.0 / 3.0)
    lam_m = d_m / d_over_lambda
    re_norm = TWO_PI * R_E_M / lam_m
    theta_b = math.asin(lam / (2.0 * d))
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, waist=waist_lambda * lam,
                  yc=0.5 * ny * dx, pol=1)
    grid = Grid(2, (nx, ny, 1), (dx, dx, 1.0), dt, (LASER, OPEN, PERIODIC),
                (OPEN, OPEN, PERIODIC), pad=3, laser=laser, re_norm=re_norm)
    q1, m1, q2, m2 = gold_ion(z_bound_neutral - free_per_ion, float(free_per_ion))
    w = 4.0 * math.pi * re_norm / d  # one column of atoms along z per site
    ion = Species(TWO_BODY, q1, m1, q2, m2, weight=w, omega_c=omega_c, a_c=0.0,
                  name="Au_preionised")
    rng = rng_for(case_id, 0)
    cx, cy = 0.5 * nx * dx, 0.5 * ny * dx
    hx, hy = 0.5 * slab[0] * dx, 0.5 * slab[1] * dx
    m = int(math.ceil(2.0 * max(hx, hy) * math.sqrt(2.0) / d)) + 2
    ii, jj = np.meshgrid(np.arange(-m, m + 1), np.arange(-m, m + 1), indexing="ij")
    a = ii.ravel() * d
    b = jj.ravel() * d
    ct, st = math.cos(theta_b), math.sin(theta_b)
    xs = cx + a * ct - b * st
    ys = cy + a * st + b * ct
    keep = (np.abs(xs - cx) < hx) & (np.abs(ys - cy) < hy)
    xs, ys = xs[keep], ys[keep]
    n_ion = xs.size
    xs = xs + rng.normal(0.0, jitter * d, n_ion)
    ys = ys + rng.normal(0.0, jitter * d, n_ion)
    ions = Particles(x=np.stack([xs, ys], axis=1), u1=np.zeros((n_ion, 3)))
    rng_e = rng_for(case_id, 1)
    lo = [int(round((cx - hx) / dx)), int(round((cy - hy) / dx))]
    hi = [lo[0] + slab[0], lo[1] + slab[1]]
    xe = stratified_positions(rng_e, lo, hi, ppc_e, grid.dx, 2)
    n_e = xe.shape[0]
    ue = rng_e.normal(0.0, thermal_sigma(t_e_ev, 1.0), size=(n_e, 3))
    w_e = free_per_ion * n_ion * w / n_e
    el = Species(POINT, -1.0, 1.0, weight=w_e, name="e_free")
    return Workload("wakefield_crystal_2d", grid, [(ion, ions), (el, Particles(x=xe, u1=ue))],
                    steps, precision,
                    notes=f"{n_ion} sites (+{free_per_ion}), {n_e} free electrons, a0={a0}")


# --------------------------------------------------------------------------
# Case 3: 3D partially ionised slab with free electrons
# --------------------------------------------------------------------------

def ionised_slab_3d(n=(512, 256, 256), ppc: int = 8, steps: int = 500, precision: int = 32,
                    omega_pb: float = 0.9, a0: float = 0.05, waist_lambda: float = 8.0,
                    cycles: int = 10, wc_range=(1.5, 4.0), nu_per_omega: float = 0.01,
                    t_ion_ev: float = 1.0, t_e_ev: float = 10.0, electrons: bool = True,
                    x_cells=None, chunk: int = 0, case_id: int = 3) -> Workload:
    """Medium filling the box between the particle walls.  x_cells = (lo, hi)
    restricts the generated particles to those x planes (chunked loading of
    the full-size case); each chunk draws from its own Philox streams."""
    dx = TWO_PI / 24.0
    dt = 0.98 * dx / math.sqrt(3.0)
    lam_m = 12.4e-9
    ny, nz = n[1], n[2]
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, waist=waist_lambda * TWO_PI,
                  yc=0.5 * ny * dx, zc=0.5 * nz * dx, pol=1)
    grid = Grid(3, tuple(n), (dx, dx, dx), dt, (LASER, PERIODIC, PERIODIC),
                (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser,
                re_norm=TWO_PI * R_E_M / lam_m)
    q1, m1, q2, m2 = gold_ion(78, 1.0)
    n_ion = bound_plasma_density(q1, m1, q2, m2, omega_pb)
    dv = dx ** 3
    w = n_ion * dv / ppc
    ion = Species(TWO_BODY, q1, m1, q2, m2, weight=w, omega_c=0.5 * sum(wc_range), a_c=0.0,
                  nu_per_omega=nu_per_omega, name="Au_q1")
    xlo, xhi = (grid.pad, n[0] - grid.pad) if x_cells is None else x_cells
    lo = [xlo, 0, 0]
    hi = [xhi, ny, nz]
    rng_i = rng_for(case_id, 2 * chunk)
    xi = stratified_positions(rng_i, lo, hi, ppc, grid.dx, 3)
    ni = xi.shape[0]
    uci = rng_i.normal(0.0, thermal_sigma(t_ion_ev, m1 + m2), size=(ni, 3))
    wci = rng_i.uniform(wc_range[0], wc_range[1], size=ni)
    species = [(ion, Particles(x=xi, u1=uci, omega_c=wci))]
    if electrons:
        ele = Species(POINT, -1.0, 1.0, weight=w, name="e")
        rng_e = rng_for(case_id, 2 * chunk + 1)
        xe = stratified_positions(rng_e, lo, hi, ppc, grid.dx, 3)
        ue = rng_e.normal(0.0, thermal_sigma(t_e_ev, 1.0), size=(xe.shape[0], 3))
        species.append((ele, Particles(x=xe, u1=ue)))
    return Workload("ionised_slab_3d", grid, species, steps, precision,
                    notes=f"{ni} two-body ions (+{ni if electrons else 0} electrons)")


def ionised_slab_3d_count(n=(512, 256, 256), ppc: int = 8, pad: int = 3) -> int:
    """Macro-ions (and, separately, free electrons) of the full slab."""
    return (n[0] - 2 * pad) * n[1] * n[2] * ppc


# --------------------------------------------------------------------------
# Case 4: mixed-precision study, Bragg geometry in 3D, 4 ions per cell
# --------------------------------------------------------------------------

def lattice_site_mean(sigma):
    """Mean over a lattice cell of the site profile exp(-(a^2 + b^2)/(2 sigma^2))
    with a, b the offsets (in lattice constants, |a|, |b| <= 1/2) from the
    nearest site: (sigma sqrt(2 pi) erf(1 / (2 sqrt(2) sigma)))^2.  Dividing
    by it keeps the mean weight at the species value."""
    return (sigma * math.sqrt(2.0 * math.pi) * math.erf(0.5 / (math.sqrt(2.0) * sigma))) ** 2


def mixed_precision_3d(n=(1024, 1024, 512), slab=(384, 640), ppc: int = 4, steps: int = 2000,
                       omega_c: float = 0.5, d_over_lambda: float = 1.5, sigma_site: float = 0.1,
                       a0: float = 1e-4, cycles: int = 20, precision: int = 32,
                       case_id: int = 4) -> Workload:
    dx = TWO_PI / 32.0
    dt = 0.98 * dx / math.sqrt(3.0)
    lam = TWO_PI
    d = d_over_lambda * lam
    d_m = (5.9e28) ** (-1.0 / 3.0)
    lam_m = d_m / d_over_lambda
    re_norm = TWO_PI * R_E_M / lam_m
    theta_b = math.asin(lam / (2.0 * d))
    laser = Laser(a0=a0, omega=1.0, t_env=cycles * TWO_PI, waist=12.0 * lam,
                  yc=0.5 * n[1] * dx, zc=0.5 * n[2] * dx, pol=1)
    grid = Grid(3, tuple(n), (dx, dx, dx), dt, (LASER, PERIODIC, PERIODIC),
                (OPEN, PERIODIC, PERIODIC), pad=3, laser=laser, re_norm=re_norm)
    q1, m1, q2, m2 = gold_ion(78, 0.0)
    # mean density one atom per d^3 = 4 pi re_norm / d^3 in units of n_c, modulated
    # by Gaussian sites of the rotated lattice so the Bragg structure survives
    n_mean = 4.0 * math.pi * re_norm / d ** 3
    dv = dx ** 3
    sp = Species(TWO_BODY, q1, m1, q2, m2, weight=n_mean * dv / ppc, omega_c=omega_c, a_c=0.0,
                 name="Au_lattice3d")
    rng = rng_for(case_id)
    lo = [max(slab[0], grid.pad), 0, 0]
    hi = [min(slab[1], n[0] - grid.pad), n[1], n[2]]
    x = stratified_positions(rng, lo, hi, ppc, grid.dx, 3)
    ct, st = math.cos(theta_b), math.sin(theta_b)
    a = x[:, 0] * ct + x[:, 1] * st
    b = -x[:, 0] * st + x[:, 1] * ct
    da = (a / d) - np.round(a / d)
    db = (b / d) - np.round(b / d)
    mod = np.exp(-(da ** 2 + db ** 2) / (2.0 * sigma_site ** 2))
    wts = sp.weight * mod / lattice_site_mean(sigma_site)
    parts = Particles(x=x, u1=np.zeros((x.shape[0], 3)), weight=wts)
    return Workload("mixed_precision_3d", grid, [(sp, parts)], steps, precision,
                    notes=f"{x.shape[0]} two-body ions, lattice-modulated weights")


WORKLOADS = {
    "neutral_medium_1d": neutral_medium_1d,
    "bragg_2d": bragg_2d,
    "ionised_slab_3d": ionised_slab_3d,
    "mixed_precision_3d": mixed_precision_3d,
    "adjoint_slab": adjoint_slab,
}


# --------------------------------------------------------------------------
# Device-side generation of the full-size 3D slab (benchmark inputs)
# --------------------------------------------------------------------------

def ionised_slab_3d_device_chunk(n=(512, 256, 256), ppc: int = 8, x_cells=(3, 35),
                                 chunk: int = 0, device="cuda", wc_range=(1.5, 4.0),
                                 t_ion_ev: float = 1.0, t_e_ev: float = 10.0,
                                 case_id: int = 3):
    """Same recipe as ionised_slab_3d for the x planes x_cells, drawn with
    torch's Philox generator on the GPU (seed = base seed + config id, offset
    by the chunk), returned as FP64 device tensors:
    (x_ion, u_c_ion, omega_c_ion, x_e, u_e), particles enumerated cell by
    cell (x fastest).  Holds no method arithmetic."""
    import torch
    dx = TWO_PI / 24.0
    q1, m1, q2, m2 = gold_ion(78, 1.0)
    ny, nz = n[1], n[2]
    out = []
    for sp in range(2):
        g = torch.Generator(device=device)
        g.manual_seed((BASE_SEED + case_id) * 1000003 + 2 * chunk + sp)
        nxc = x_cells[1] - x_cells[0]
        m = nxc * ny * nz * ppc
        p = torch.arange(m, device=device, dtype=torch.int64)
        cell = p // ppc
        sub = (p % ppc).to(torch.float64)
        cx = (cell % nxc).to(torch.float64) + x_cells[0]
        rem = cell // nxc
        cy = (rem % ny).to(torch.float64)
        cz = (rem // ny).to(torch.float64)
        x = torch.empty((m, 3), device=device, dtype=torch.float64)
        x[:, 0] = (cx + (sub + torch.rand(m, generator=g, device=device,
                                          dtype=torch.float64)) / ppc) * dx
        x[:, 1] = (cy + torch.rand(m, generator=g, device=device, dtype=torch.float64)) * dx
        x[:, 2] = (cz + torch.rand(m, generator=g, device=device, dtype=torch.float64)) * dx
        del p, cell, sub, cx, cy, cz, rem
        if sp == 0:
            u = torch.randn((m, 3), generator=g, device=device, dtype=torch.float64)
            u *= thermal_sigma(t_ion_ev, m1 + m2)
            wc = torch.rand(m, generator=g, device=device, dtype=torch.float64)
            wc = wc_range[0] + (wc_range[1] - wc_range[0]) * wc
            out += [x, u, wc]
        else:
            u = torch.randn((m, 3), generator=g, device=device, dtype=torch.float64)
            u *= thermal_sigma(t_e_ev, 1.0)
            out += [x, u]
    return tuple(out)


def mixed_precision_3d_device_chunk(n=(1024, 1024, 512), ppc: int = 4, x_cells=(384, 400),
                                    chunk: int = 0, device="cuda", d_over_lambda: float = 1.5,
                                    sigma_site: float = 0.1, case_id: int = 4):
    """Same recipe as mixed_precision_3d for the x planes x_cells, drawn with
    torch's Philox generator on the GPU (seed = base seed + config id, offset
    by the chunk), as FP64 device tensors (x, weight / species weight),
    particles enumerated cell by cell (x fastest), at rest.  Holds no method
    arithmetic."""
    import torch
    dx = TWO_PI / 32.0
    lam = TWO_PI
    d = d_over_lambda * lam
    theta_b = math.asin(lam / (2.0 * d))
    ny, nz = n[1], n[2]
    g = torch.Generator(device=device)
    g.manual_seed((BASE_SEED + case_id) * 1000003 + chunk)
    nxc = x_cells[1] - x_cells[0]
    m = nxc * ny * nz * ppc
    p = torch.arange(m, device=device, dtype=torch.int64)
    cell = p // ppc
    sub = (p % ppc).to(torch.float64)
    cx = (cell % nxc).to(torch.float64) + x_cells[0]
    rem = cell // nxc
    cy = (rem % ny).to(torch.float64)
    cz = (rem // ny).to(torch.float64)
    del p, cell, rem
    x = torch.empty((m, 3), device=device, dtype=torch.float64)
    x[:, 0] = (cx + (sub + torch.rand(m, generator=g, device=device, dtype=torch.float64))
               / ppc) * dx
    x[:, 1] = (cy + torch.rand(m, generator=g, device=device, dtype=torch.float64)) * dx
    x[:, 2] = (cz + torch.rand(m, generator=g, device=device, dtype=torch.float64)) * dx
    del cx, cy, cz, sub
    ct, st = math.cos(theta_b), math.sin(theta_b)
    a = (x[:, 0] * ct + x[:, 1] * st) / d
    b = (-x[:, 0] * st + x[:, 1] * ct) / d
    a -= torch.round(a)
    b -= torch.round(b)
    w = torch.exp(-(a * a + b * b) / (2.0 * sigma_site ** 2)) / lattice_site_mean(sigma_site)
    del a, b
    return x, w
