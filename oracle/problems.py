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


def spt_slab(case, dims=None):
    """Space-parameter-time heat slab on dims (x, y, z, P, r, k, t) (Sec. 2.3:
    parameters as extra tensor dimensions; Sec. 2.5: their 1D integrals, the
    conductivity entering through the k-weighted mass int Ntilde_i k Ntilde_j dk):
      rho c_p  M M M M M M   G
      1        K M M M M W^k M   (and the y and z stiffness terms alike)
    Source 2 eta P / (pi r^2 d_v) exp(-2 ((x - x0(t))^2 + (y - y0)^2) / r^2)
    1(H - z <= d_v): linear in P, interpolated nodally in t and in r (the
    reading used for time, applied to the radius), so load term (j, l) has
    x-factor 2 eta / (pi r_l^2 d_v) exp(-2 (x - x0(t_j))^2 / r_l^2), y-factor
    exp(-2 (y - y0)^2 / r_l^2), z-factor the top layer, P-factor P, r-factor
    Ntilde_l, k-factor 1, t-factor Ntilde_j."""
    dims = dims or dims_of(case)
    dx, dy, dz, dP, dr, dk, dt = dims
    mats = [
        {"mass": dx.matrix("mass"), "stiff": dx.matrix("stiff")},
        {"mass": dy.matrix("mass"), "stiff": dy.matrix("stiff")},
        {"mass": dz.matrix("mass"), "stiff": dz.matrix("stiff")},
        {"mass": dP.matrix("mass")},
        {"mass": dr.matrix("mass")},
        {"mass": dk.matrix("mass"), "wmass": dk.matrix("wmass", coef=lambda k: k)},
        {"mass": dt.matrix("mass"), "ddt": dt.matrix("ddt")},
    ]
    terms = [
        (case.rho_cp_per_ms, ("mass", "mass", "mass", "mass", "mass", "mass", "ddt")),
        (1.0, ("stiff", "mass", "mass", "mass", "mass", "wmass", "mass")),
        (1.0, ("mass", "stiff", "mass", "mass", "mass", "wmass", "mass")),
        (1.0, ("mass", "mass", "stiff", "mass", "mass", "wmass", "mass")),
    ]
    tn, rn = dt.nodes, dr.nodes
    nt, nr = len(tn), len(rn)
    x0 = case.x_start + case.speed * tn
    cols_x = []
    for j in range(nt):
        for l in range(nr):
            amp = 2.0 * case.eta / (np.pi * rn[l] ** 2 * case.depth)
            cols_x.append(dx.load(lambda x, c=x0[j], r2=rn[l] ** 2, a=amp: a * np.exp(-2.0 * (x - c) ** 2 / r2)))
    Fx = np.stack(cols_x, axis=1)
    Fy = np.stack([dy.load(lambda y, r2=r ** 2: np.exp(-2.0 * (y - case.y0) ** 2 / r2)) for r in rn], axis=1)
    H = case.height
    Fz = dz.load(lambda z: (H - z <= case.depth).astype(np.float64))[:, None]
    FP = dP.load(lambda P: P)[:, None]
    Fr = mats[4]["mass"].toarray()
    Fk = dk.load(lambda k: np.ones_like(k))[:, None]
    Ft = mats[6]["mass"].toarray()
    jj, ll = np.meshgrid(np.arange(nt), np.arange(nr), indexing="ij")
    jj, ll = jj.reshape(-1), ll.reshape(-1)          # load term q = j * nr + l
    zero = np.zeros(nt * nr, np.int64)
    cols = [jj * nr + ll, ll, zero, zero, ll, zero, jj]
    return SeparatedProblem(mats, terms, [Fx, Fy, Fz, FP, Fr, Fk, Ft], cols, [D.fixed for D in dims])


def spt_polynomial(case, dims=None):
    """Same space-parameter-time operator with the load of the exact field
    u = z (2H - z) t P (zero at z = 0 and t = 0, zero flux on every other
    face, polynomial of degree <= 2 in each dim): f = rho c_p z (2H - z) P
    + 2 k t P, two separable terms."""
    dims = dims or dims_of(case)
    mats = spt_slab(case, dims).mats
    dx, dy, dz, dP, dr, dk, dt = dims
    H = case.height
    one = lambda v: np.ones_like(v)
    F = [dx.loads([one, one]), dy.loads([one, one]),
         dz.loads([lambda z: case.rho_cp_per_ms * z * (2 * H - z), one]),
         dP.loads([lambda P: P, lambda P: P]), dr.loads([one, one]),
         dk.loads([one, lambda k: 2.0 * k]), dt.loads([one, lambda t: t])]
    terms = spt_slab_terms(case)
    return SeparatedProblem(mats, terms, F, [np.arange(2)] * 7, [D.fixed for D in dims])


def spt_slab_terms(case):
    return [
        (case.rho_cp_per_ms, ("mass", "mass", "mass", "mass", "mass", "mass", "ddt")),
        (1.0, ("stiff", "mass", "mass", "mass", "mass", "wmass", "mass")),
        (1.0, ("mass", "stiff", "mass", "mass", "mass", "wmass", "mass")),
        (1.0, ("mass", "mass", "stiff", "mass", "mass", "wmass", "mass")),
    ]


# ---------------------------------------------------------------------------
# Space-time convergence problem (first results section): exact field
# u = a(t) exp(-y^2) exp(-(x - c(t))^2), a = 1 - exp(-decay t), c = speed t + x0,
# rho c_p = k = 1.  The source is derived here from u (the printed one does
# not belong to this u): with xi = x - c,
#   du/dt  = exp(-y^2 - xi^2) [decay exp(-decay t) + 2 speed a xi]
#   u_xx   = a exp(-y^2 - xi^2) (4 xi^2 - 2),  u_yy = a exp(-y^2 - xi^2) (4 y^2 - 2)
#   f = du/dt - u_xx - u_yy
#     = exp(-y^2) exp(-xi^2) [decay e^{-decay t} + 2 speed a xi + a (2 - 4 xi^2)]
#       + a exp(-xi^2) exp(-y^2) (2 - 4 y^2).
# Separated form: nodal interpolation in time (load term pair per time node
# t_j), and the boundary data by a nodal lifting (below).


def st_exact(case, x, y, t):
    a = 1.0 - np.exp(-case.decay * t)
    return a * np.exp(-y ** 2 - (x - case.speed * t - case.x0) ** 2)


def st_source(case, x, y, t):
    a = 1.0 - np.exp(-case.decay * t)
    xi = x - case.speed * t - case.x0
    g = np.exp(-y ** 2 - xi ** 2)
    return g * (case.decay * np.exp(-case.decay * t) + 2.0 * case.speed * a * xi + a * (2.0 - 4.0 * xi ** 2)
                + a * (2.0 - 4.0 * y ** 2))


def st_lift_terms(case, dims):
    """Nodal lifting of the face data as separable terms (sign, [nodal vector
    per dim]).  With g the nodal interpolant of u^ex -- per time node j the
    rank-one term a_j exp(-(x - c_j)^2) (x) exp(-y^2) (x) 1 (x) e_j -- and
    chi_d the indicator of the interior nodes of a spatial dim, the lifting
    g - (chi_x g_x)(chi_y g_y)(chi_z g_z) e_j equals u^ex at every boundary
    node and 0 at every interior node."""
    dx, dy, dz, dt = dims
    out = []
    for j, tj in enumerate(dt.nodes):
        a = 1.0 - np.exp(-case.decay * tj)
        gx = a * np.exp(-(dx.nodes - case.speed * tj - case.x0) ** 2)
        gy = np.exp(-dy.nodes ** 2)
        gz = np.ones(dz.n)
        et = np.zeros(dt.n)
        et[j] = 1.0
        vecs = [gx, gy, gz]
        masked = []
        for D, v in zip((dx, dy, dz), vecs):
            w = v.copy()
            w[list(D.fixed)] = 0.0
            masked.append(w)
        out.append((1.0, vecs + [et]))
        out.append((-1.0, masked + [et.copy()]))
    return out


def st_convergence(case, dims=None):
    """The homogeneous part u_0 = u - u_lift: a(u_0, v) = l(v) - a(u_lift, v),
    u_0 = 0 on every spatial face and at t = 0.  Load terms: per time node two
    source terms, and per lifting term and operator term one term
    -sign gamma prod_d A_d v_d."""
    dims = dims or dims_of(case)
    dx, dy, dz, dt = dims
    mats = [{"mass": D.matrix("mass"), "stiff": D.matrix("stiff")} for D in (dx, dy, dz)]
    mats.append({"mass": dt.matrix("mass"), "ddt": dt.matrix("ddt")})
    terms = [(1.0, ("mass", "mass", "mass", "ddt")), (1.0, ("stiff", "mass", "mass", "mass")),
             (1.0, ("mass", "stiff", "mass", "mass")), (1.0, ("mass", "mass", "stiff", "mass"))]
    cols = [[], [], [], []]
    Mt = mats[3]["mass"].toarray()
    for j, tj in enumerate(dt.nodes):
        a = 1.0 - np.exp(-case.decay * tj)
        c = case.speed * tj + case.x0
        fa = lambda x, a=a, c=c, tj=tj: np.exp(-(x - c) ** 2) * (
            case.decay * np.exp(-case.decay * tj) + 2.0 * case.speed * a * (x - c) + a * (2.0 - 4.0 * (x - c) ** 2))
        fb = lambda x, a=a, c=c: a * np.exp(-(x - c) ** 2)
        for fx, fy in ((fa, lambda y: np.exp(-y ** 2)), (fb, lambda y: (2.0 - 4.0 * y ** 2) * np.exp(-y ** 2))):
            cols[0].append(dx.load(fx))
            cols[1].append(dy.load(fy))
            cols[2].append(dz.load(lambda z: np.ones_like(z)))
            cols[3].append(Mt[:, j])
    for sign, vecs in st_lift_terms(case, dims):
        for gamma, names in terms:
            col = [mats[d][names[d]] @ vecs[d] for d in range(4)]
            col[0] = -sign * gamma * col[0]
            for d in range(4):
                cols[d].append(np.asarray(col[d]).ravel())
    F = [np.stack(c, axis=1) for c in cols]
    R = F[0].shape[1]
    return SeparatedProblem(mats, terms, F, [np.arange(R)] * 4, [D.fixed for D in dims])


def st_field_factors(case, dims, U):
    """Factors of the full field u = u_0 + u_lift (rank M + 2 n_t)."""
    lift = st_lift_terms(case, dims)
    out = [np.array(u, copy=True) for u in U]
    for d in range(4):
        cols = [sign * vecs[d] if d == 0 else vecs[d] for sign, vecs in lift]
        out[d] = np.concatenate([out[d], np.stack(cols, axis=1)], axis=1)
    return out


# ---------------------------------------------------------------------------
# Space-parameter-time convergence problem on eight dimensions (second
# results section): u = rho c_p P a(k, t) E(x) E(y), a = 1 - exp(-decay k t),
# E(v) = exp(-width v^2), with  rho c_p du/dt - k lap u = f:
#   du/dt = rho c_p P decay k exp(-decay k t) E E
#   lap u = rho c_p P a (E''(x) E(y) + E(x) E''(y)),  E'' = E (4 width^2 v^2 - 2 width)
#   f = decay rho^2 c_p^2 P k exp(-decay k t) E E
#       + rho c_p P k a [E (2 width - 4 width^2 x^2) E + E E (2 width - 4 width^2 y^2)]
# (width 25: 2 width - 4 width^2 v^2 = 50 (1 - 50 v^2), the printed source).
# Operator terms on (x, y, z, k, P, rho, c_p, t): rho c_p M..M W^rho W^cp G,
# and k K_x / K_y / K_z with W^k; nodal interpolation in t for the source and
# the lifting.


def spt8_exact(case, x, y, k, P, rho, cp, t):
    return rho * cp * P * (1.0 - np.exp(-case.decay * k * t)) * np.exp(-case.width * (x ** 2 + y ** 2))


def spt8_terms():
    w = ("mass", "mass", "mass", "mass", "mass", "wmass", "wmass", "ddt")
    return [
        (1.0, w),
        (1.0, ("stiff", "mass", "mass", "wmass", "mass", "mass", "mass", "mass")),
        (1.0, ("mass", "stiff", "mass", "wmass", "mass", "mass", "mass", "mass")),
        (1.0, ("mass", "mass", "stiff", "wmass", "mass", "mass", "mass", "mass")),
    ]


def spt8_mats(dims):
    dx, dy, dz, dk, dP, dr, dc, dt = dims
    lin = lambda v: v
    return [
        {"mass": dx.matrix("mass"), "stiff": dx.matrix("stiff")},
        {"mass": dy.matrix("mass"), "stiff": dy.matrix("stiff")},
        {"mass": dz.matrix("mass"), "stiff": dz.matrix("stiff")},
        {"mass": dk.matrix("mass"), "wmass": dk.matrix("wmass", coef=lin)},
        {"mass": dP.matrix("mass")},
        {"mass": dr.matrix("mass"), "wmass": dr.matrix("wmass", coef=lin)},
        {"mass": dc.matrix("mass"), "wmass": dc.matrix("wmass", coef=lin)},
        {"mass": dt.matrix("mass"), "ddt": dt.matrix("ddt")},
    ]


def spt8_lift_terms(case, dims):
    """Nodal lifting (sign, [nodal vector per dim]) as for the space-time
    problem: per time node the nodal interpolant of u^ex, once whole and once
    with its interior spatial nodes (in x, y and z) removed, subtracted."""
    dx, dy, dz, dk, dP, dr, dc, dt = dims
    E = lambda v: np.exp(-case.width * v ** 2)
    out = []
    for j, tj in enumerate(dt.nodes):
        et = np.zeros(dt.n)
        et[j] = 1.0
        vecs = [E(dx.nodes), E(dy.nodes), np.ones(dz.n), 1.0 - np.exp(-case.decay * dk.nodes * tj),
                dP.nodes.copy(), dr.nodes.copy(), dc.nodes.copy(), et]
        masked = [v.copy() for v in vecs]
        for d, D in enumerate((dx, dy, dz)):
            masked[d][list(D.fixed)] = 0.0
        out.append((1.0, vecs))
        out.append((-1.0, masked))
    return out


def spt8_convergence(case, dims=None):
    """Homogeneous part u_0 = u - u_lift with u_0 = 0 on every spatial face and
    at t = 0: load = source (three terms per time node) - a(u_lift, .)."""
    dims = dims or dims_of(case)
    dx, dy, dz, dk, dP, dr, dc, dt = dims
    mats = spt8_mats(dims)
    terms = spt8_terms()
    wd = case.width
    E = lambda v: np.exp(-wd * v ** 2)
    E2 = lambda v: np.exp(-wd * v ** 2) * (2.0 * wd - 4.0 * wd * wd * v ** 2)
    Mt = mats[7]["mass"].toarray()
    cols = [[] for _ in range(8)]
    for j, tj in enumerate(dt.nodes):
        src = [
            (case.decay, [E, E, None, lambda k: k * np.exp(-case.decay * k * tj), lambda P: P,
                          lambda r: r ** 2, lambda c: c ** 2]),
            (1.0, [E2, E, None, lambda k: k * (1.0 - np.exp(-case.decay * k * tj)), lambda P: P,
                   lambda r: r, lambda c: c]),
            (1.0, [E, E2, None, lambda k: k * (1.0 - np.exp(-case.decay * k * tj)), lambda P: P,
                   lambda r: r, lambda c: c]),
        ]
        for coef, fs in src:
            for d, (D, f) in enumerate(zip(dims[:7], fs)):
                col = D.load(f if f is not None else (lambda v: np.ones_like(v)))
                cols[d].append(coef * col if d == 0 else col)
            cols[7].append(Mt[:, j])
    for sign, vecs in spt8_lift_terms(case, dims):
        for gamma, names in terms:
            for d in range(8):
                col = np.asarray(mats[d][names[d]] @ vecs[d]).ravel()
                cols[d].append(-sign * gamma * col if d == 0 else col)
    F = [np.stack(c, axis=1) for c in cols]
    R = F[0].shape[1]
    return SeparatedProblem(mats, terms, F, [np.arange(R)] * 8, [D.fixed for D in dims])


def spt8_field_factors(case, dims, U):
    """Factors of u = u_0 + u_lift."""
    lift = spt8_lift_terms(case, dims)
    out = []
    for d in range(8):
        cols = [sign * vecs[d] if d == 0 else vecs[d] for sign, vecs in lift]
        out.append(np.concatenate([np.asarray(U[d]), np.stack(cols, axis=1)], axis=1))
    return out
