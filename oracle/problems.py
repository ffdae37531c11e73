"""Term tables and separated loads of the paper's PDEs (oracle).

Sec. 2.4: the transient heat equation  rho c_p du/dt - div(k grad u) = f  with
the moving Gaussian volumetric source, read with the readings listed below,
and the Poisson operator of the PDE-examples table (Sec. 2.4) for the steady case.  Each PDE becomes a sum of
separable terms (one 1D matrix per dimension) and a sum of separable loads.

Readings:
  * heat source depth indicator: the laser heats the top layer of thickness
    d_v, i.e. 1(H - z <= d_v) (the printed indicator 1(z >= d_v) would heat the
    bulk);
  * the moving source is not separable in (x, t); it is interpolated in time
    with the same 1D C-HiDeNN basis, exact at time nodes by the Kronecker-delta
    property:  f(x, y, z, t) ~ sum_j Ntilde_j(t) f(x, y, z, t_j).  Load term j
    then has x-factor A exp(-2 (x - x0(t_j))^2 / r^2), y-factor
    exp(-2 (y - y0)^2 / r^2), z-factor 1(H - z <= d_v) and t-factor Ntilde_j(t),
    whose 1D integral is column j of the time mass matrix;
  * scan path x0(t) = x_start + v t, y0 fixed.
"""
import numpy as np

from .assemble import Dim1D
from .separated import SeparatedProblem


def dims_of(case):
    return [Dim1D(ax.nodes(), ax.s, ax.a, ax.p, ax.n_gauss, ax.fixed) for ax in case.axes]


def poisson2d(case, dims=None):
    """-lap u = 2 pi^2 sin(pi x) sin(pi y) + 2x(1-x) + 2y(1-y) on [0,1]^2, u = 0 on the boundary."""
    dims = dims or dims_of(case)
    mats = [{"mass": D.matrix("mass"), "stiff": D.matrix("stiff")} for D in dims]
    terms = [(1.0, ("stiff", "mass")), (1.0, ("mass", "stiff"))]
    pi = np.pi
    fx = [lambda x: 2 * pi * pi * np.sin(pi * x), lambda x: 2 * x * (1 - x), lambda x: np.ones_like(x)]
    fy = [lambda y: np.sin(pi * y), lambda y: np.ones_like(y), lambda y: 2 * y * (1 - y)]
    F = [dims[0].loads(fx), dims[1].loads(fy)]
    cols = [np.arange(3), np.arange(3)]
    return SeparatedProblem(mats, terms, F, cols, [D.fixed for D in dims])


def poisson2d_exact(x, y):
    return np.sin(np.pi * x) * np.sin(np.pi * y) + x * (1 - x) * y * (1 - y)


def poisson2d_polynomial(dims):
    """-lap u = 2y(1-y) + 2x(1-x): exact solution u = x(1-x) y(1-y) (rank one)."""
    mats = [{"mass": D.matrix("mass"), "stiff": D.matrix("stiff")} for D in dims]
    terms = [(1.0, ("stiff", "mass")), (1.0, ("mass", "stiff"))]
    fx = [lambda x: 2 * x * (1 - x), lambda x: np.ones_like(x)]
    fy = [lambda y: np.ones_like(y), lambda y: 2 * y * (1 - y)]
    F = [dims[0].loads(fx), dims[1].loads(fy)]
    return SeparatedProblem(mats, terms, F, [np.arange(2), np.arange(2)], [D.fixed for D in dims])


def spacetime_polynomial(dx, dt):
    """du/dt - d2u/dx2 = x(1-x) + 2t on [0,1] x [0,T]: exact u = x(1-x) t,
    u = 0 at x = 0, 1 and at t = 0 (space-time, time-derivative term)."""
    mats = [{"mass": dx.matrix("mass"), "stiff": dx.matrix("stiff")},
            {"mass": dt.matrix("mass"), "ddt": dt.matrix("ddt")}]
    terms = [(1.0, ("mass", "ddt")), (1.0, ("stiff", "mass"))]
    fx = [lambda x: x * (1 - x), lambda x: np.ones_like(x)]
    ft = [lambda t: np.ones_like(t), lambda t: 2 * t]
    F = [dx.loads(fx), dt.loads(ft)]
    return SeparatedProblem(mats, terms, F, [np.arange(2), np.arange(2)], [dx.fixed, dt.fixed])


def heat_source_amplitude(case):
    """2 eta P / (pi r^2 d_v) in W/mm^3 (Sec. 2.4, moving-source equation)."""
    return 2.0 * case.eta * case.power / (np.pi * case.radius ** 2 * case.depth)


def heat_operator(case, dims):
    """1D matrices and term table of rho c_p du/dt - k (u_xx + u_yy + u_zz)
    on dims (x, y, z, t): rho c_p M(x)M(y)M(z)G(t) + k [K M M M + M K M M + M M K M]."""
    dx, dy, dz, dt = dims
    mats = [
        {"mass": dx.matrix("mass"), "stiff": dx.matrix("stiff")},
        {"mass": dy.matrix("mass"), "stiff": dy.matrix("stiff")},
        {"mass": dz.matrix("mass"), "stiff": dz.matrix("stiff")},
        {"mass": dt.matrix("mass"), "ddt": dt.matrix("ddt")},
    ]
    rc, k = case.rho_cp_per_ms, case.k
    terms = [
        (rc, ("mass", "mass", "mass", "ddt")),
        (k, ("stiff", "mass", "mass", "mass")),
        (k, ("mass", "stiff", "mass", "mass")),
        (k, ("mass", "mass", "stiff", "mass")),
    ]
    return mats, terms


def heat_slab(case, dims=None):
    """One space-time slab of the heat equation (dims x, y, z, t) with the
    time-interpolated moving Gaussian source."""
    dims = dims or dims_of(case)
    dx, dy, dz, dt = dims
    mats, terms = heat_operator(case, dims)
    amp = heat_source_amplitude(case)
    r2 = case.radius ** 2
    tn = dt.nodes
    x0 = case.x_start + case.speed * tn
    Fx = np.stack([dx.load(lambda x, c=c: amp * np.exp(-2.0 * (x - c) ** 2 / r2)) for c in x0], axis=1)
    Fy = dy.load(lambda y: np.exp(-2.0 * (y - case.y0) ** 2 / r2))[:, None]
    H = case.height
    Fz = dz.load(lambda z: (H - z <= case.depth).astype(np.float64))[:, None]
    Ft = mats[3]["mass"].toarray()          # column j = int Ntilde_i Ntilde_j dt
    nt = len(tn)
    cols = [np.arange(nt), np.zeros(nt, np.int64), np.zeros(nt, np.int64), np.arange(nt)]
    return SeparatedProblem(mats, terms, [Fx, Fy, Fz, Ft], cols, [D.fixed for D in dims])


def heat_polynomial(case, dims=None):
    """Same operator with the load of the exact field u = z (2H - z) t: u = 0 at
    z = 0 and t = 0, zero flux on every other face, so
    f = rho c_p z (2H - z) + 2 k t (two separable terms)."""
    dims = dims or dims_of(case)
    dx, dy, dz, dt = dims
    mats, terms = heat_operator(case, dims)
    H = case.height
    one = lambda v: np.ones_like(v)
    Fx = dx.loads([one, one])
    Fy = dy.loads([one, one])
    Fz = dz.loads([lambda z: case.rho_cp_per_ms * z * (2 * H - z), one])
    Ft = dt.loads([one, lambda t: 2.0 * case.k * t])
    cols = [np.arange(2)] * 4
    return SeparatedProblem(mats, terms, [Fx, Fy, Fz, Ft], cols, [D.fixed for D in dims])
