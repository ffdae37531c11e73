"""Seeded synthetic inputs for the TAPS slab solve.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
only sizes, physical constants, grid coordinates and seeded random draws: no
step of the method's arithmetic (basis, quadrature, assembly, contraction,
solve) lives here, so both implementations build their own problem from these
plain numbers.

Workloads (shaped after the paper's additive-manufacturing heat problems):

* ``poisson2d``   -- 2D steady Poisson, -lap u = f on [0,1]^2, homogeneous
  Dirichlet on every side, manufactured f = 2 pi^2 sin(pi x) sin(pi y)
  + 2x(1-x) + 2y(1-y) (exact u = sin sin + x(1-x)y(1-y)).
* ``heat_slab``   -- one space-time slab of the transient heat equation
  rho c_p du/dt - k lap u = f on 1 mm x 1 mm x 0.2 mm with a moving Gaussian
  volumetric source (paper Sec. 2.4, moving-source equation), homogeneous
  initial condition and u = 0 on the bottom face z = 0, other faces adiabatic.
* ``heat_slab_batch`` -- uneven batch of heat slabs with random grid sizes and
  random (P, r, k, y0) draws.

Units: lengths in mm, time in ms, power in W, so k is W/(mm K), rho*c_p is
J/(mm^3 K) and the source amplitude is W/mm^3; the time derivative carries the
factor 1e3 (ms -> s) inside ``rho_cp_per_ms``.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np


@dataclass(frozen=True)
class Axis:
    """One tensor dimension: a uniform grid plus the C-HiDeNN hyperparameters."""

    name: str
    lo: float
    hi: float
    n: int
    s: int = 2          # patch size
    a: float = 20.0     # dilation
    p: int = 2          # reproducing order
    n_gauss: int = 5    # Gauss points per element
    fixed: Tuple[int, ...] = ()  # node indices held at zero

    def nodes(self) -> np.ndarray:
        return np.linspace(self.lo, self.hi, self.n)


@dataclass(frozen=True)
class Poisson2D:
    axes: Tuple[Axis, Axis]
    M: int
    seed: int
    kind: str = "poisson2d"


@dataclass(frozen=True)
class HeatSlab:
    """Parameters of one space-time slab (x, y, z, t)."""

    axes: Tuple[Axis, Axis, Axis, Axis]
    M: int
    seed: int
    k: float = 0.020          # W/(mm K)   (20 W/(m K))
    rho_cp: float = 4.0e-3    # J/(mm^3 K) (8000 kg/m^3 * 500 J/(kg K))
    eta: float = 0.4
    power: float = 200.0      # W
    radius: float = 0.050     # mm
    depth: float = 0.050      # mm, penetration depth d_v
    speed: float = 1.0        # mm/ms (1 m/s)
    x_start: float = 0.1      # mm
    y0: float = 0.5           # mm
    kind: str = "heat_slab"

    @property
    def rho_cp_per_ms(self) -> float:
        """rho*c_p in J/(mm^3 K) times d/dt in 1/ms -> W/(mm^3 K) scale."""
        return self.rho_cp * 1.0e3

    @property
    def height(self) -> float:
        return self.axes[2].hi


def poisson2d(n_el: int = 64, M: int = 10, seed: int = 0, s: int = 2,
              a: float = 20.0, p: int = 2, n_gauss: int = 5) -> Poisson2D:
    n = n_el + 1
    ax = lambda nm: Axis(nm, 0.0, 1.0, n, s, a, p, n_gauss, fixed=(0, n - 1))
    return Poisson2D((ax("x"), ax("y")), M, seed)


def heat_slab(nx: int = 512, ny: int = 512, nz: int = 128, nt: int = 257,
              M: int = 40, seed: int = 2, s: int = 2, a: float = 20.0,
              p: int = 2, n_gauss: int = 5, duration_ms: float = 0.8,
              **phys) -> HeatSlab:
    """The single-slab transient heat workload (default: 512x512x128 x 257)."""
    ax = [
        Axis("x", 0.0, 1.0, nx, s, a, p, n_gauss),
        Axis("y", 0.0, 1.0, ny, s, a, p, n_gauss),
        Axis("z", 0.0, 0.2, nz, s, a, p, n_gauss, fixed=(0,)),
        Axis("t", 0.0, duration_ms, nt, s, a, p, n_gauss, fixed=(0,)),
    ]
    return HeatSlab(tuple(ax), M, seed, **phys)


def heat_slab_batch(batch: int = 64, n_lo: int = 64, n_hi: int = 1024,
                    M: int = 30, seed: int = 3, nt_hi: int | None = None):
    """Uneven batch of heat slabs: every grid size drawn from U{n_lo..n_hi};
    power, radius, conductivity and track offset drawn per problem."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(batch):
        nx, ny, nz, nt = (int(v) for v in rng.integers(n_lo, n_hi + 1, size=4))
        if nt_hi is not None:
            nt = min(nt, nt_hi)
        P = float(rng.uniform(100.0, 300.0))
        r = float(rng.uniform(0.030, 0.080))
        k = float(rng.uniform(0.010, 0.030))
        y0 = float(rng.uniform(0.3, 0.7))
        out.append(heat_slab(nx, ny, nz, nt, M=M, seed=seed * 100003 + b,
                             power=P, radius=r, k=k, y0=y0))
    return out


def heat_slab_family(batch: int = 64, seed: int = 4, **grid):
    """Independent heat slabs on one grid (default 512x512x128x257, M=40):
    per slab power, radius, conductivity and track offset drawn like the uneven
    batch, so the slabs stand for parameter queries or separate tracks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(batch):
        P = float(rng.uniform(100.0, 300.0))
        r = float(rng.uniform(0.030, 0.080))
        k = float(rng.uniform(0.010, 0.030))
        y0 = float(rng.uniform(0.3, 0.7))
        out.append(heat_slab(seed=seed * 100003 + b, power=P, radius=r, k=k, y0=y0, **grid))
    return out


@dataclass(frozen=True)
class SPTSlab:
    """One space-parameter-time slab (x, y, z, P, r, k, t): the heat slab with
    laser power P, beam radius r and conductivity k as extra tensor
    dimensions of uniform nodes over their ranges (paper Sec. 2.3, the
    space-parameter-time variables)."""

    axes: Tuple[Axis, Axis, Axis, Axis, Axis, Axis, Axis]
    M: int
    seed: int
    rho_cp: float = 4.0e-3
    eta: float = 0.4
    depth: float = 0.050
    speed: float = 1.0
    x_start: float = 0.1
    y0: float = 0.5
    kind: str = "spt_slab"

    @property
    def rho_cp_per_ms(self) -> float:
        return self.rho_cp * 1.0e3

    @property
    def height(self) -> float:
        return self.axes[2].hi


PARAM_BOUNDS = {"P": (100.0, 300.0), "r": (0.030, 0.080), "k": (0.010, 0.030)}


def spt_slab(nx: int, ny: int, nz: int, nt: int, n_param: int = 32, M: int = 30, seed: int = 3,
             s: int = 2, p: int = 2, duration_ms: float = 0.8, **phys) -> SPTSlab:
    """Space-parameter-time slab: x, y in [0, 1 mm], z in [0, 0.2 mm], P, r, k
    on n_param uniform nodes of their ranges, t in [0, duration]; z = 0 and
    t = 0 fixed."""
    ax = [
        Axis("x", 0.0, 1.0, nx, s, 20.0, p),
        Axis("y", 0.0, 1.0, ny, s, 20.0, p),
        Axis("z", 0.0, 0.2, nz, s, 20.0, p, fixed=(0,)),
        Axis("P", *PARAM_BOUNDS["P"], n_param, s, 20.0, p),
        Axis("r", *PARAM_BOUNDS["r"], n_param, s, 20.0, p),
        Axis("k", *PARAM_BOUNDS["k"], n_param, s, 20.0, p),
        Axis("t", 0.0, duration_ms, nt, s, 20.0, p, fixed=(0,)),
    ]
    return SPTSlab(tuple(ax), M, seed, **phys)


def spt_batch(batch: int = 64, n_lo: int = 64, n_hi: int = 1024, n_param: int = 32, M: int = 30,
              seed: int = 3):
    """Uneven batch of space-parameter-time slabs: n_x, n_y, n_z, n_t drawn
    from U{n_lo..n_hi}, the track offset y0 from U[0.3, 0.7] mm per problem."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(batch):
        nx, ny, nz, nt = (int(v) for v in rng.integers(n_lo, n_hi + 1, size=4))
        y0 = float(rng.uniform(0.3, 0.7))
        out.append(spt_slab(nx, ny, nz, nt, n_param=n_param, M=M, seed=seed * 100003 + b, y0=y0))
    return out


@dataclass(frozen=True)
class STConvergence:
    """The space-time convergence problem of the paper's first results
    section: du/dt - lap u = f with rho c_p = k = 1 and the exact field
    u = (1 - exp(-decay t)) exp(-y^2 - (x - speed t - x0)^2) (independent of
    z), u = 0 at t = 0 and u = u^ex on every spatial face.  Readings (the
    paper gives neither): x in [0, 10], y in [-5, 5], z in [0, 1], t in
    [0, 0.05], so the Gaussian travels from x = 5 onto the x = 10 face (the
    faces carry O(1) data there and on both z faces)."""

    axes: Tuple[Axis, Axis, Axis, Axis]
    M: int
    seed: int
    speed: float = 100.0
    x0: float = 5.0
    decay: float = 15.0
    kind: str = "st_convergence"


def st_convergence(n: int = 100, nt: int = 100, M: int = 25, s: int = 1, p: int = 1, seed: int = 5,
                   n_y: int | None = None, n_z: int | None = None, T: float = 0.05) -> STConvergence:
    """n nodes along x (and y, z unless given), nt along t; every spatial face
    Dirichlet (fixed rows of the homogeneous part), t = 0 fixed."""
    ny = n if n_y is None else n_y
    nz = n if n_z is None else n_z
    ends = lambda m: (0, m - 1)
    ax = [
        Axis("x", 0.0, 10.0, n, s, 20.0, p, fixed=ends(n)),
        Axis("y", -5.0, 5.0, ny, s, 20.0, p, fixed=ends(ny)),
        Axis("z", 0.0, 1.0, nz, s, 20.0, p, fixed=ends(nz)),
        Axis("t", 0.0, T, nt, s, 20.0, p, fixed=(0,)),
    ]
    return STConvergence(tuple(ax), M, seed)


@dataclass(frozen=True)
class SPT8Convergence:
    """The space-parameter-time convergence problem of the paper's second
    results section on eight dimensions (x, y, z, k, P, rho, c_p, t):
    rho c_p du/dt - k lap u = f with the exact field
    u = rho c_p P (1 - exp(-decay k t)) exp(-width (x^2 + y^2)) (independent
    of z), u = 0 at t = 0, u = u^ex on every spatial face.  Readings (the
    paper states neither domain nor ranges): x, y in [-1, 1], z in [0, 1],
    k, P, rho, c_p in [1, 2], t in [0, 0.2]."""

    axes: Tuple[Axis, ...]
    M: int
    seed: int
    decay: float = 15.0
    width: float = 25.0
    kind: str = "spt8_convergence"


def spt8_convergence(n: int = 20, M: int = 20, s: int = 1, p: int = 1, seed: int = 8,
                     n_param: int | None = None, nt: int | None = None) -> SPT8Convergence:
    """n nodes along every dim (n_param along k, P, rho, c_p and nt along t
    when given); every spatial face Dirichlet, t = 0 fixed."""
    npar = n if n_param is None else n_param
    ntt = n if nt is None else nt
    ends = lambda m: (0, m - 1)
    ax = [
        Axis("x", -1.0, 1.0, n, s, 20.0, p, fixed=ends(n)),
        Axis("y", -1.0, 1.0, n, s, 20.0, p, fixed=ends(n)),
        Axis("z", 0.0, 1.0, n, s, 20.0, p, fixed=ends(n)),
        Axis("k", 1.0, 2.0, npar, s, 20.0, p),
        Axis("P", 1.0, 2.0, npar, s, 20.0, p),
        Axis("rho", 1.0, 2.0, npar, s, 20.0, p),
        Axis("cp", 1.0, 2.0, npar, s, 20.0, p),
        Axis("t", 0.0, 0.2, ntt, s, 20.0, p, fixed=(0,)),
    ]
    return SPT8Convergence(tuple(ax), M, seed)


@dataclass(frozen=True)
class NonlinearHeat:
    """Space-time heat problem with temperature-dependent material (paper's
    third results section and the appendix on solution-dependent
    coefficients): d/dt (rho c_p(u) u) - div (k(u) grad u) = f with the linear
    fits k(u) = m_k u + n_k and rho c_p(u) = m_c u + n_c the paper gives
    (Inconel 718; u read as the temperature rise above ambient, mm, s, W, J).
    u = 0 on the left and right faces (x = 0, x = L_x) and at t = 0, zero flux
    elsewhere.  Source: the moving Gaussian beam of radius r at speed v,
    volumetric through the plate thickness (2 eta P / (pi r^2 H)
    exp(-2 ((x - x0 - v t)^2 + (y - y0)^2) / r^2)), or, with
    source="poly", the load of the exact field u = a x (L_x - x) t."""

    axes: Tuple[Axis, Axis, Axis, Axis]
    M: int
    seed: int
    m_k: float = 1.52e-5
    n_k: float = 5.29e-3
    m_c: float = 6.11e-7
    n_c: float = 3.25e-3
    power: float = 100.0
    eta: float = 0.4
    radius: float = 0.5
    speed: float = 500.0
    x_start: float = 1.0
    y0: float = 5.0
    amp: float = 1.0
    source: str = "gauss"
    kind: str = "nonlinear_heat"


def nonlinear_heat(nx: int = 101, ny: int = 101, nz: int = 11, nt: int = 126, M: int = 10, seed: int = 9,
                   Lx: float = 10.0, Ly: float = 10.0, H: float = 1.0, T: float = 0.02, s: int = 2, p: int = 2,
                   **phys) -> NonlinearHeat:
    """The paper's nonlinear set-up by default: 10 mm x 10 mm x 1 mm, beam
    radius 0.5 mm at 500 mm/s, 10 elements per beam diameter in x and y, time
    increment 1.6e-4 s over 0.02 s."""
    ax = [
        Axis("x", 0.0, Lx, nx, s, 20.0, p, fixed=(0, nx - 1)),
        Axis("y", 0.0, Ly, ny, s, 20.0, p),
        Axis("z", 0.0, H, nz, s, 20.0, p),
        Axis("t", 0.0, T, nt, s, 20.0, p, fixed=(0,)),
    ]
    return NonlinearHeat(tuple(ax), M, seed, **phys)


def multitrack_slabs(steps_per_slab: int, n_slabs: int, n: int = 301, M: int | None = None, seed: int = 11,
                     hatch: float = 0.05, tracks: int = 1, L: float = 1.5, H: float = 1.5, h_mesh: float = 0.005,
                     s: int = 2, p: int = 2, x_margin: float = 0.1):
    """Space-time slabs of the multi-track LPBF set-up (paper table of
    multi-track parameters; Ti-6Al-4V table): 1.5 mm cube, 5 um mesh (301
    nodes per spatial dim), P = 200 W, r = 50 um, v = 500 mm/s, eta = 0.25,
    penetration depth 50 um, hatch 50 um, k = 22 W/(m K), rho c_p = 4270 kg/m^3
    x 745 J/(kg K).  Reading (not stated): one time step moves the beam one
    mesh cell (dt = h / v = 10 us), and M = 5 x time steps per slab (the
    paper's single-track rule) capped at 48.  Tracks run in alternating
    directions along x, y0 = L/2 - (tracks - 1) hatch / 2 + j hatch; slab T
    starts where slab T-1 ended.  Returns the slab cases in order."""
    dt = h_mesh / 0.5              # ms (v = 0.5 mm/ms)
    T_slab = steps_per_slab * dt
    nt = steps_per_slab + 1
    M = min(48, 5 * steps_per_slab) if M is None else M
    track_len = L - 2 * x_margin
    slabs_per_track = max(1, int(round(track_len / (0.5 * T_slab))))
    out = []
    for T in range(n_slabs):
        j, k = divmod(T, slabs_per_track)
        j = j % tracks
        y0 = L / 2 - (tracks - 1) * hatch / 2 + j * hatch
        fwd = j % 2 == 0
        x0 = x_margin + 0.5 * T_slab * k if fwd else L - x_margin - 0.5 * T_slab * k
        ax = [
            Axis("x", 0.0, L, n, s, 20.0, p),
            Axis("y", 0.0, L, n, s, 20.0, p),
            Axis("z", 0.0, H, n, s, 20.0, p, fixed=(0,)),
            Axis("t", 0.0, T_slab, nt, s, 20.0, p, fixed=(0,)),
        ]
        out.append(HeatSlab(tuple(ax), M, seed * 1009 + T, k=0.022, rho_cp=4.27e-6 * 745.0, eta=0.25,
                            power=200.0, radius=0.05, depth=0.05, speed=0.5 if fwd else -0.5, x_start=x0, y0=y0))
    return out


def initial_factors(axes, M: int, seed: int):
    """Random initial mode factors U_d ~ N(0,1) (n_d x M, float64, row-major),
    one PCG64 stream per problem, dims drawn in order; rows of fixed nodes are 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Us = []
    for ax in axes:
        U = rng.standard_normal((ax.n, M))
        if ax.fixed:
            U[list(ax.fixed), :] = 0.0
        Us.append(np.ascontiguousarray(U))
    return Us


def output_points(ax: Axis, n_pts: int) -> np.ndarray:
    """Uniform evaluation points spanning an axis (end points included)."""
    return np.linspace(ax.lo, ax.hi, n_pts)


def shrink(case, factor: int):
    """Same workload on a grid coarsened by ``factor`` along every axis
    (fixed nodes remapped), for oracle-sized parity runs."""
    axes = []
    for ax in case.axes:
        n = max(2 * ax.s + 2, (ax.n - 1) // factor + 1)
        fixed = tuple(sorted({0 if f == 0 else n - 1 for f in ax.fixed}))
        axes.append(replace(ax, n=n, fixed=fixed))
    return replace(case, axes=tuple(axes))


def mlp_init(widths, seed: int = 0):
    """Seeded initial weights of the warm-start network: W_l ~ N(0, 2 / in)
    (out x in), zero biases; float64 arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = [rng.standard_normal((o, i)) * np.sqrt(2.0 / i) for i, o in zip(widths[:-1], widths[1:])]
    bs = [np.zeros(o) for o in widths[1:]]
    return Ws, bs


def large_slab(n: int = 15000, nz: int = 15, nt: int = 513, M: int = 60, seed: int = 5,
               width_mm: float = 15.0, duration_ms: float = 1.0, s: int = 2, a: float = 20.0, p: int = 2,
               n_gauss: int = 5, **phys) -> HeatSlab:
    """The large single slab: x, y in [0, 15 mm] with 15000 nodes each (about
    1 um spacing), z in [0, 0.2 mm] with 15 nodes, t in [0, 1 ms] with 513
    nodes (512 steps), M = 60; the moving source and material of the heat
    slab, the track centred in y."""
    ax = [
        Axis("x", 0.0, width_mm, n, s, a, p, n_gauss),
        Axis("y", 0.0, width_mm, n, s, a, p, n_gauss),
        Axis("z", 0.0, 0.2, nz, s, a, p, n_gauss, fixed=(0,)),
        Axis("t", 0.0, duration_ms, nt, s, a, p, n_gauss, fixed=(0,)),
    ]
    phys.setdefault("y0", 0.5 * width_mm)
    return HeatSlab(tuple(ax), M, seed, **phys)
