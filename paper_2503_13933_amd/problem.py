"""Device-side problem set-up for the library (argument marshalling).

Builds a ``taps_problem_t`` for a workload description: node coordinates go to
the device, then the library computes Gauss points (taps_gauss_points), source
factors at those points (taps_source1d) and the 1D bands and load columns
(taps_assemble1d).  The term tables written here are the separated forms of
the paper's PDEs (Sec. 2.4-2.5):

  heat slab (x, y, z, t):  rho c_p M M M G  +  k (K M M M + M K M M + M M K M)
  Poisson 2D (x, y):       K M + M K

with the moving Gaussian source interpolated in time by the C-HiDeNN basis
(load term j = beam centred at x0(t_j) times Ntilde_j(t)).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import capi
from .capi import Basis1D, Problem

F64 = torch.float64


class _Grid:
    """Grid-only data of one axis, shared by every problem built on that grid
    with the same matrix kinds: nodes, Gauss rule, shape values at the Gauss
    points, the 1D bands, the fixed-row mask, and load matrices that depend
    on the grid alone (keyed by the caller).  Read-only once built."""

    def __init__(self, h, ax, kinds, device):
        self.x = torch.tensor(ax.nodes(), dtype=F64, device=device)
        self.basis = Basis1D(ax.n, self.x.data_ptr(), ax.s, float(ax.a), ax.p, ax.n_gauss)
        ngp = (ax.n - 1) * ax.n_gauss
        self.xg = torch.empty(ngp, dtype=F64, device=device)
        self.wg = torch.empty(ngp, dtype=F64, device=device)
        capi.taps_gauss_points(h, self.basis, self.xg, self.wg)
        self.Ng = torch.empty((ngp, 2 * ax.s + 2), dtype=F64, device=device)
        self.firstg = torch.empty(ngp, dtype=torch.int32, device=device)
        capi.taps_shape1d(h, self.basis, self.xg, self.Ng, None, self.firstg)
        self.band = torch.empty((len(kinds), ax.n, 4 * ax.s + 3), dtype=F64, device=device)
        capi.taps_assemble1d(h, self.basis, list(kinds), self.band)
        self.fixed = torch.zeros(ax.n, dtype=torch.uint8, device=device)
        if ax.fixed:
            self.fixed[list(ax.fixed)] = 1
        self.loads = {}


def _grid(h, ax, kinds, device):
    cache = h.__dict__.setdefault("_grids", {})
    key = (ax.lo, ax.hi, ax.n, ax.s, float(ax.a), ax.p, ax.n_gauss, tuple(ax.fixed), tuple(kinds), str(device))
    g = cache.get(key)
    if g is None:
        g = cache[key] = _Grid(h, ax, kinds, device)
    return g


class DeviceAxis:
    """Nodes, basis descriptor, Gauss rule and bands of one dimension.

    shared=True takes the grid-only data from the handle's cache (computed
    once per grid and kinds, never written afterwards), so only the loads are
    assembled per problem (taps_load1d); problems whose bands are rewritten
    later (the coefficient problems of Algorithm 2) use their own."""

    def __init__(self, h, ax, kinds, device, shared=False):
        self.ax = ax
        self.n = ax.n
        self.kinds = list(kinds)
        self.F = None
        self.h = h
        self.device = device
        self.ngp = (ax.n - 1) * ax.n_gauss
        self.grid = _grid(h, ax, kinds, device) if shared else None
        if self.grid is not None:
            g = self.grid
            self.x, self.basis, self.xg, self.wg, self.band, self.fixed = g.x, g.basis, g.xg, g.wg, g.band, g.fixed
            return
        self.x = torch.tensor(ax.nodes(), dtype=F64, device=device)
        self.basis = Basis1D(ax.n, self.x.data_ptr(), ax.s, float(ax.a), ax.p, ax.n_gauss)
        self.xg = torch.empty(self.ngp, dtype=F64, device=device)
        self.wg = torch.empty(self.ngp, dtype=F64, device=device)
        capi.taps_gauss_points(h, self.basis, self.xg, self.wg)
        self.band = torch.empty((len(kinds), ax.n, 4 * ax.s + 3), dtype=F64, device=device)
        self.fixed = torch.zeros(ax.n, dtype=torch.uint8, device=device)
        if ax.fixed:
            self.fixed[list(ax.fixed)] = 1

    def source(self, kind, params, n_cols=1, centers=None):
        """Source factor(s) at the Gauss points, (n_cols, ngp)."""
        out = torch.empty((n_cols, self.ngp), dtype=F64, device=self.device)
        basis = self.basis if kind == capi.SRC_NODAL else None
        capi.taps_source1d(self.h, kind, self.xg, n_cols, params, out, centers=centers, basis=basis)
        return out

    def assemble(self, f_g, coef_g=None):
        """Bands of self.kinds and load columns of f_g ((R, ngp) at the Gauss
        points); coef_g: the weighted-mass coefficient at the Gauss points.
        On a shared grid only the loads are assembled."""
        f_g = f_g.contiguous()
        R = f_g.shape[0]
        self.F = torch.empty((self.n, R), dtype=F64, device=self.device)
        if self.grid is not None:
            assert coef_g is None, "a shared grid's bands are fixed"
            g, ax = self.grid, self.ax
            capi.taps_load1d(self.h, ax.n, ax.s, ax.n_gauss, g.Ng, g.firstg, g.wg, f_g, self.F)
            return self
        capi.taps_assemble1d(self.h, self.basis, self.kinds, self.band, coef_g=coef_g, f_g=f_g, F=self.F, n_loads=R)
        return self

    def assemble_shared(self, key, make_f_g):
        """Loads that depend on the grid alone (e.g. the nodal time loads):
        assembled once per shared grid and key, then the same tensor for every
        problem on it (read-only)."""
        if self.grid is None:
            return self.assemble(make_f_g())
        F = self.grid.loads.get(key)
        if F is None:
            self.assemble(make_f_g())
            self.grid.loads[key] = self.F
        else:
            self.F = F
        return self


class DeviceProblem:
    """A taps_problem_t plus the device tensors it points to."""

    def __init__(self, h, axes, terms, load_cols, M):
        self.h = h
        self.axes = axes
        self.M = M
        self.D = len(axes)
        self.keep = []
        p = Problem()
        p.D, p.M, p.T = self.D, M, len(terms)
        given = [len(c) for c in load_cols if c is not None]
        R = given[0] if given else axes[0].F.shape[1]
        p.R = R
        for d, a in enumerate(axes):
            p.n[d] = a.n
            p.s[d] = a.ax.s
            p.n_kinds[d] = len(a.kinds)
            p.d_band[d] = a.band.data_ptr()
            p.R_cols[d] = a.F.shape[1]
            p.d_F[d] = a.F.data_ptr()
            p.d_fixed[d] = a.fixed.data_ptr()
            cols = load_cols[d]
            if cols is not None and len(cols) == a.F.shape[1] and np.array_equal(cols, np.arange(len(cols))):
                cols = None     # the identity map: one load column per term, no grouping
            if cols is None:
                assert a.F.shape[1] == R
                continue
            cols = np.asarray(cols, dtype=np.int32)
            order = np.argsort(cols, kind="stable").astype(np.int32)
            ptr = np.searchsorted(cols[order], np.arange(a.F.shape[1] + 1)).astype(np.int32)
            for arr, field in ((cols, "d_load_col"), (ptr, "d_load_ptr"), (order, "d_load_idx")):
                t = torch.tensor(arr, dtype=torch.int32, device=a.device)
                self.keep.append(t)
                getattr(p, field)[d] = t.data_ptr()
        for t, (gamma, kinds) in enumerate(terms):
            p.gamma[t] = gamma
            for d, k in enumerate(kinds):
                p.term_kind[t][d] = k
        self.struct = p
        self.R = R

    def factors(self, Us):
        """Device copies of host factors (list of n_d x M arrays)."""
        return [torch.tensor(np.ascontiguousarray(U), dtype=F64, device=self.axes[0].device) for U in Us]


def heat_slab(h, case, device="cuda", M=None):
    """Device problem of one heat slab (workload taps_workloads.HeatSlab)."""
    M = case.M if M is None else M
    ax, ay, az, at = case.axes
    # grid-only data (shape values, bands, the nodal time loads) computed once
    # per grid on the handle and shared by every slab on it
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device, shared=True)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device, shared=True)
    Z = DeviceAxis(h, az, [capi.MASS, capi.STIFF], device, shared=True)
    T = DeviceAxis(h, at, [capi.MASS, capi.DDT], device, shared=True)
    amp = 2.0 * case.eta * case.power / (math.pi * case.radius ** 2 * case.depth)
    centers = torch.tensor(case.x_start + case.speed * at.nodes(), dtype=F64, device=device)
    X.assemble(X.source(capi.SRC_GAUSS, [amp, case.radius], n_cols=at.n, centers=centers))
    yc = torch.tensor([case.y0], dtype=F64, device=device)
    Y.assemble(Y.source(capi.SRC_GAUSS, [1.0, case.radius], n_cols=1, centers=yc))
    Z.assemble(Z.source(capi.SRC_TOPLAYER, [case.height, case.depth]))
    T.assemble_shared(("nodal",), lambda: T.source(capi.SRC_NODAL, [], n_cols=at.n))
    rc, k = case.rho_cp_per_ms, case.k
    terms = [(rc, (0, 0, 0, 1)), (k, (1, 0, 0, 0)), (k, (0, 1, 0, 0)), (k, (0, 0, 1, 0))]
    zeros = np.zeros(at.n, dtype=np.int32)
    prob = DeviceProblem(h, [X, Y, Z, T], terms, [None, zeros, zeros, None], M)
    prob.keep.append(centers)
    prob.keep.append(yc)
    return prob


def heat_polynomial(h, case, device="cuda", M=None):
    """Heat operator with the load of u = z (2H - z) t (exactly representable, rank one)."""
    M = case.M if M is None else M
    ax, ay, az, at = case.axes
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device)
    Z = DeviceAxis(h, az, [capi.MASS, capi.STIFF], device)
    T = DeviceAxis(h, at, [capi.MASS, capi.DDT], device)
    H, rc, k = case.height, case.rho_cp_per_ms, case.k
    one = lambda A: A.source(capi.SRC_POLY, [1.0])
    X.assemble(torch.cat([one(X), one(X)]))
    Y.assemble(torch.cat([one(Y), one(Y)]))
    Z.assemble(torch.cat([Z.source(capi.SRC_POLY, [0.0, 2.0 * H * rc, -rc]), one(Z)]))
    T.assemble(torch.cat([one(T), T.source(capi.SRC_POLY, [0.0, 2.0 * k])]))
    terms = [(rc, (0, 0, 0, 1)), (k, (1, 0, 0, 0)), (k, (0, 1, 0, 0)), (k, (0, 0, 1, 0))]
    return DeviceProblem(h, [X, Y, Z, T], terms, [None] * 4, M)


def poisson2d(h, case, device="cuda", M=None):
    """-lap u = 2 pi^2 sin(pi x) sin(pi y) + 2x(1-x) + 2y(1-y), u = 0 on the boundary."""
    M = case.M if M is None else M
    ax, ay = case.axes
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device)
    pi = math.pi
    X.assemble(torch.cat([X.source(capi.SRC_SIN, [2 * pi * pi, pi]), X.source(capi.SRC_POLY, [0.0, 2.0, -2.0]),
                          X.source(capi.SRC_POLY, [1.0])]))
    Y.assemble(torch.cat([Y.source(capi.SRC_SIN, [1.0, pi]), Y.source(capi.SRC_POLY, [1.0]),
                          Y.source(capi.SRC_POLY, [0.0, 2.0, -2.0])]))
    terms = [(1.0, (1, 0)), (1.0, (0, 1))]
    return DeviceProblem(h, [X, Y], terms, [None, None], M)


def _spt_axes(h, case, device):
    ax, ay, az, aP, ar, ak, at = case.axes
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device)
    Z = DeviceAxis(h, az, [capi.MASS, capi.STIFF], device)
    Pd = DeviceAxis(h, aP, [capi.MASS], device)
    Rd = DeviceAxis(h, ar, [capi.MASS], device)
    Kd = DeviceAxis(h, ak, [capi.MASS, capi.WMASS], device)
    T = DeviceAxis(h, at, [capi.MASS, capi.DDT], device)
    return X, Y, Z, Pd, Rd, Kd, T


# rho c_p M M M M M M G, then k (K M M | M K M | M M K) M M W^k M
SPT_TERMS_KINDS = [(0, 0, 0, 0, 0, 0, 1), (1, 0, 0, 0, 0, 1, 0), (0, 1, 0, 0, 0, 1, 0), (0, 0, 1, 0, 0, 1, 0)]


def spt_slab(h, case, device="cuda", M=None):
    """Device problem of a space-parameter-time slab (x, y, z, P, r, k, t):
    P, r, k as tensor dimensions, k entering through the k-weighted mass; the
    source linear in P and interpolated nodally in t and r (load term
    j * n_r + l)."""
    M = case.M if M is None else M
    X, Y, Z, Pd, Rd, Kd, T = _spt_axes(h, case, device)
    at, ar = case.axes[6], case.axes[4]
    nt, nr = at.n, ar.n
    rn = ar.nodes()
    centers = torch.tensor(case.x_start + case.speed * at.nodes(), dtype=F64, device=device)
    yc = torch.tensor([case.y0], dtype=F64, device=device)
    fx = torch.stack([X.source(capi.SRC_GAUSS, [2.0 * case.eta / (math.pi * r * r * case.depth), float(r)],
                               n_cols=nt, centers=centers) for r in rn], dim=1)      # (nt, nr, ngp)
    X.assemble(fx.reshape(nt * nr, X.ngp))
    del fx
    Y.assemble(torch.cat([Y.source(capi.SRC_GAUSS, [1.0, float(r)], n_cols=1, centers=yc) for r in rn]))
    Z.assemble(Z.source(capi.SRC_TOPLAYER, [case.height, case.depth]))
    Pd.assemble(Pd.source(capi.SRC_POLY, [0.0, 1.0]))
    Rd.assemble(Rd.source(capi.SRC_NODAL, [], n_cols=nr))
    Kd.assemble(Kd.source(capi.SRC_POLY, [1.0]), coef_g=Kd.source(capi.SRC_POLY, [0.0, 1.0])[0].contiguous())
    T.assemble(T.source(capi.SRC_NODAL, [], n_cols=nt))
    q = np.arange(nt * nr)
    jj, ll, zero = q // nr, q % nr, np.zeros(nt * nr, dtype=np.int32)
    cols = [q, ll, zero, zero, ll, zero, jj]
    terms = [(case.rho_cp_per_ms if t == 0 else 1.0, kinds) for t, kinds in enumerate(SPT_TERMS_KINDS)]
    prob = DeviceProblem(h, [X, Y, Z, Pd, Rd, Kd, T], terms, cols, M)
    prob.keep += [centers, yc]
    return prob


def spt_polynomial(h, case, device="cuda", M=None):
    """Space-parameter-time operator with the load of u = z (2H - z) t P
    (exactly representable, rank one): f = rho c_p z (2H - z) P + 2 k t P."""
    M = case.M if M is None else M
    X, Y, Z, Pd, Rd, Kd, T = _spt_axes(h, case, device)
    H, rc = case.height, case.rho_cp_per_ms
    one = lambda A: A.source(capi.SRC_POLY, [1.0])
    for A in (X, Y, Rd):
        A.assemble(torch.cat([one(A), one(A)]))
    Z.assemble(torch.cat([Z.source(capi.SRC_POLY, [0.0, 2.0 * H * rc, -rc]), one(Z)]))
    Pd.assemble(torch.cat([Pd.source(capi.SRC_POLY, [0.0, 1.0])] * 2))
    kc = Kd.source(capi.SRC_POLY, [0.0, 1.0])[0].contiguous()
    Kd.assemble(torch.cat([one(Kd), Kd.source(capi.SRC_POLY, [0.0, 2.0])]), coef_g=kc)
    T.assemble(torch.cat([one(T), T.source(capi.SRC_POLY, [0.0, 1.0])]))
    terms = [(rc if t == 0 else 1.0, kinds) for t, kinds in enumerate(SPT_TERMS_KINDS)]
    return DeviceProblem(h, [X, Y, Z, Pd, Rd, Kd, T], terms, [None] * 7, M)


def _expquad(h, pts, rows, device):
    """EXPQUAD source columns at points: rows = list of 8-coefficient tuples."""
    coef = torch.tensor(np.asarray(rows, dtype=np.float64).reshape(-1), dtype=F64, device=device)
    out = torch.empty((len(rows), pts.numel()), dtype=F64, device=device)
    capi.taps_source1d(h, capi.SRC_EXPQUAD, pts, len(rows), [], out, centers=coef)
    return out


class STProblem(DeviceProblem):
    """The space-time convergence problem's homogeneous part u_0 plus the
    device factors of its nodal lifting (to add to u_0's factors for the
    full field)."""

    def lift_factors(self):
        return self.lift

    def full_factors(self, U):
        """Factors of u = u_0 + u_lift (rank M + 2 n_t), device tensors."""
        return [torch.cat([u, l], dim=1).contiguous() for u, l in zip(U, self.lift)]


def st_convergence(h, case, device="cuda", M=None):
    """Device problem of the space-time convergence study (exact field
    a(t) exp(-y^2 - (x - c(t))^2), rho c_p = k = 1), solved for the
    homogeneous part u_0 = u - u_lift:  a(u_0, v) = l(v) - a(u_lift, v).
    Source (derived from the exact field, nodal in time): per time node j
    the terms exp(-(x-c_j)^2)[decay e^{-decay t_j} + 2 speed a_j xi +
    a_j (2 - 4 xi^2)] e^{-y^2} and a_j exp(-(x-c_j)^2) (2 - 4 y^2) e^{-y^2}.
    Lifting: per time node g_j - (chi g_j) (the nodal interpolant of the
    exact field minus its interior part), each entering the load as
    -sign gamma_tau prod_d A^tau_d v_d for the four operator terms."""
    M = case.M if M is None else M
    ax, ay, az, at = case.axes
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device)
    Z = DeviceAxis(h, az, [capi.MASS, capi.STIFF], device)
    T = DeviceAxis(h, at, [capi.MASS, capi.DDT], device)
    tn = at.nodes()
    nt = at.n
    a = 1.0 - np.exp(-case.decay * tn)
    c = case.speed * tn + case.x0
    rows_a = [(c[j], 1.0, 0.0, case.decay * np.exp(-case.decay * tn[j]) + 2.0 * a[j], 2.0 * case.speed * a[j],
               -4.0 * a[j], 0.0, 0.0) for j in range(nt)]
    rows_b = [(c[j], 1.0, 0.0, a[j], 0.0, 0.0, 0.0, 0.0) for j in range(nt)]
    # source load terms, ordered (j, A), (j, B)
    fx = torch.stack([_expquad(h, X.xg, rows_a, device), _expquad(h, X.xg, rows_b, device)], dim=1)
    gy = _expquad(h, Y.xg, [(0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0), (0.0, 1.0, 0.0, 2.0, 0.0, -4.0, 0.0, 0.0)],
                  device)
    fy = gy.unsqueeze(0).expand(nt, 2, Y.ngp)
    ones = lambda A: A.source(capi.SRC_POLY, [1.0])
    fz = ones(Z).expand(2 * nt, Z.ngp)
    ft = T.source(capi.SRC_NODAL, [], n_cols=nt).unsqueeze(1).expand(nt, 2, T.ngp)
    for A, f in ((X, fx), (Y, fy), (Z, fz), (T, ft)):
        A.assemble(f.reshape(2 * nt, A.ngp).contiguous())
    # lifting vectors at the nodes (n_d x n_t, one column per time node), full and interior-masked
    vx = _expquad(h, X.x, rows_b, device).T.contiguous()
    vy = _expquad(h, Y.x, [(0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0)], device).T.expand(ay.n, nt).contiguous()
    vz = torch.ones((az.n, nt), dtype=F64, device=device)
    vt = torch.eye(nt, dtype=F64, device=device)
    full = [vx, vy, vz, vt]
    masked = []
    for A, v in zip((X, Y, Z), full[:3]):
        w = v.clone()
        w[list(A.ax.fixed)] = 0.0
        masked.append(w)
    masked.append(vt)
    terms = [(1.0, (0, 0, 0, 1)), (1.0, (1, 0, 0, 0)), (1.0, (0, 1, 0, 0)), (1.0, (0, 0, 1, 0))]
    axes = [X, Y, Z, T]
    n_lift = 2 * len(terms) * nt
    Fs = []
    for d, A in enumerate(axes):
        F = torch.empty((A.n, 2 * nt + n_lift), dtype=F64, device=device)
        F[:, :2 * nt] = A.F
        col = 2 * nt
        for sign, vecs in ((1.0, full), (-1.0, masked)):
            for gamma, kinds in terms:
                alpha = -sign * gamma if d == 0 else 1.0
                capi.taps_band_apply(h, A.ax.s, A.band[kinds[d]], vecs[d], F[:, col:col + nt], alpha=alpha)
                col += nt
        Fs.append(F)
    for A, F in zip(axes, Fs):
        A.F = F
    prob = STProblem(h, axes, terms, [None] * 4, M)
    # lifting factors of the full field: g_j and -(chi g_j) per time node
    prob.lift = [torch.cat([vx, -masked[0]], dim=1), torch.cat([vy, masked[1]], dim=1),
                 torch.cat([vz, masked[2]], dim=1), torch.cat([vt, vt], dim=1)]
    return prob


def spt8_convergence(h, case, device="cuda", M=None):
    """Device problem of the eight-dimensional space-parameter-time
    convergence study (x, y, z, k, P, rho, c_p, t; exact field
    rho c_p P (1 - exp(-decay k t)) exp(-width (x^2 + y^2))), solved for the
    homogeneous part u_0 = u - u_lift.  Operator: rho c_p M..M W^rho W^cp G
    and k K / W^k in each spatial dim.  Source (derived from the exact field,
    nodal in time): per time node
      decay * E(x) E(y) 1 (k e^{-decay k t_j}) P rho^2 c_p^2,
      E2(x) E(y) 1 (k (1 - e^{-decay k t_j})) P rho c_p  and  E(x) E2(y) ...,
    E = exp(-width v^2), E2 = E (2 width - 4 width^2 v^2).  Lifting as for the
    space-time problem (per time node the nodal interpolant of the exact
    field, whole and with its interior spatial nodes removed)."""
    M = case.M if M is None else M
    ax, ay, az, ak, aP, ar, ac, at = case.axes
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device)
    Z = DeviceAxis(h, az, [capi.MASS, capi.STIFF], device)
    K = DeviceAxis(h, ak, [capi.MASS, capi.WMASS], device)
    Pd = DeviceAxis(h, aP, [capi.MASS], device)
    Rd = DeviceAxis(h, ar, [capi.MASS, capi.WMASS], device)
    Cd = DeviceAxis(h, ac, [capi.MASS, capi.WMASS], device)
    T = DeviceAxis(h, at, [capi.MASS, capi.DDT], device)
    axes = [X, Y, Z, K, Pd, Rd, Cd, T]
    tn, nt, wd, dc = at.nodes(), at.n, case.width, case.decay
    E = (0.0, wd, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0)
    E2 = (0.0, wd, 0.0, 2.0 * wd, 0.0, -4.0 * wd * wd, 0.0, 0.0)
    poly = lambda A, c: A.source(capi.SRC_POLY, c)
    # source terms ordered (j, term)
    fx = torch.stack([_expquad(h, X.xg, [E], device)[0] * dc, _expquad(h, X.xg, [E2], device)[0],
                      _expquad(h, X.xg, [E], device)[0]])
    fy = torch.stack([_expquad(h, Y.xg, [E], device)[0], _expquad(h, Y.xg, [E], device)[0],
                      _expquad(h, Y.xg, [E2], device)[0]])
    rows_k = []
    for j in range(nt):
        lam = -dc * tn[j]
        rows_k += [(0.0, 0.0, lam, 0.0, 1.0, 0.0, 0.0, 0.0), (0.0, 0.0, lam, 0.0, -1.0, 0.0, 0.0, 1.0),
                   (0.0, 0.0, lam, 0.0, -1.0, 0.0, 0.0, 1.0)]
    fk = _expquad(h, K.xg, rows_k, device)
    src = {
        0: fx.unsqueeze(0).expand(nt, 3, X.ngp), 1: fy.unsqueeze(0).expand(nt, 3, Y.ngp),
        2: poly(Z, [1.0]).expand(3 * nt, Z.ngp), 3: fk,
        4: poly(Pd, [0.0, 1.0]).expand(3 * nt, Pd.ngp),
        5: torch.stack([poly(Rd, [0.0, 0.0, 1.0])[0], poly(Rd, [0.0, 1.0])[0], poly(Rd, [0.0, 1.0])[0]])
        .unsqueeze(0).expand(nt, 3, Rd.ngp),
        6: torch.stack([poly(Cd, [0.0, 0.0, 1.0])[0], poly(Cd, [0.0, 1.0])[0], poly(Cd, [0.0, 1.0])[0]])
        .unsqueeze(0).expand(nt, 3, Cd.ngp),
        7: T.source(capi.SRC_NODAL, [], n_cols=nt).unsqueeze(1).expand(nt, 3, T.ngp),
    }
    lin = {3: K, 5: Rd, 6: Cd}
    for d, A in enumerate(axes):
        coef = poly(A, [0.0, 1.0])[0].contiguous() if d in lin else None
        A.assemble(src[d].reshape(3 * nt, A.ngp).contiguous(), coef_g=coef)
    # lifting vectors at the nodes, one column per time node
    ones = lambda A: torch.ones((A.n, nt), dtype=F64, device=device)
    vx = _expquad(h, X.x, [E], device).T.expand(ax.n, nt).contiguous()
    vy = _expquad(h, Y.x, [E], device).T.expand(ay.n, nt).contiguous()
    vk = _expquad(h, K.x, [(0.0, 0.0, -dc * tn[j], -1.0, 0.0, 0.0, 1.0, 0.0) for j in range(nt)], device).T.contiguous()
    vP = Pd.x[:, None].expand(aP.n, nt).contiguous()
    vr = Rd.x[:, None].expand(ar.n, nt).contiguous()
    vc = Cd.x[:, None].expand(ac.n, nt).contiguous()
    vt = torch.eye(nt, dtype=F64, device=device)
    full = [vx, vy, ones(Z), vk, vP, vr, vc, vt]
    masked = [v.clone() for v in full]
    for d, A in enumerate((X, Y, Z)):
        masked[d][list(A.ax.fixed)] = 0.0
    kinds = [(0, 0, 0, 0, 0, 1, 1, 1), (1, 0, 0, 1, 0, 0, 0, 0), (0, 1, 0, 1, 0, 0, 0, 0), (0, 0, 1, 1, 0, 0, 0, 0)]
    terms = [(1.0, k) for k in kinds]
    n_lift = 2 * len(terms) * nt
    for d, A in enumerate(axes):
        F = torch.empty((A.n, 3 * nt + n_lift), dtype=F64, device=device)
        F[:, :3 * nt] = A.F
        col = 3 * nt
        for sign, vecs in ((1.0, full), (-1.0, masked)):
            for gamma, kk in terms:
                alpha = -sign * gamma if d == 0 else 1.0
                capi.taps_band_apply(h, A.ax.s, A.band[kk[d]], vecs[d], F[:, col:col + nt], alpha=alpha)
                col += nt
        A.F = F
    prob = STProblem(h, axes, terms, [None] * 8, M)
    prob.lift = [torch.cat([full[d] if d else full[0], -masked[0] if d == 0 else masked[d]], dim=1).contiguous()
                 for d in range(8)]
    return prob


def build(h, case, device="cuda", M=None):
    if case.kind == "heat_slab":
        return heat_slab(h, case, device, M)
    if case.kind == "spt_slab":
        return spt_slab(h, case, device, M)
    if case.kind == "st_convergence":
        return st_convergence(h, case, device, M)
    if case.kind == "spt8_convergence":
        return spt8_convergence(h, case, device, M)
    if case.kind == "poisson2d":
        return poisson2d(h, case, device, M)
    raise ValueError(case.kind)
