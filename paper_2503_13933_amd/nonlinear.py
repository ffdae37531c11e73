"""Solution-dependent material coefficients: the global-local loop of the
paper's Algorithm 2 (driver above the C ABI; every numeric step runs in the
library's kernels).

With the linear fits k(u) = m_k u + n_k and rho c_p(u) = m_c u + n_c the
coefficients are in TD form whenever u is.  Each global stage freezes them
and solves the linear problem
    int v d/dt (c u) + int grad v . k grad u = int v f
by Algorithm 1 (taps_als); the local stage rebuilds the coefficients from
the new u: u is compressed to R_c modes by the paper's mode compression
(Algorithm 1 on the mass-only operator with u as load, taps_band_apply for
the loads M_d U_d, fixed rows kept) and the coefficient modes enter the next
operator as weighted 1D matrices (taps_assemble1d kinds WMASS, WSTIFF and
WDDT with the mode's values and, in time, derivative at the Gauss points,
from taps_shape1d and taps_interp1d).  Operator terms per global stage:
    n_c (M, M, M, G),  m_c (W[v_x], W[v_y], W[v_z], W_G[v_t])  per mode v,
    n_k (K, M, M, M) + (M, K, M, M) + (M, M, K, M),
    m_k (W_K[v_x], W[v_y], W[v_z], W[v_t]) and its y, z analogues per mode.
The loop stops when the compressed field changes by at most tol > 0 in the
mass norm between global stages (taps_td_inner); tol = 0 runs every outer
stage (the change has a rounding floor near 1e-8 and can read exactly 0).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import capi
from .problem import F64, DeviceAxis, DeviceProblem


def _gauss_values(h, A, V):
    """Values and derivatives of the columns of V (n x R) at the axis's Gauss
    points: (R, ngp) each."""
    L = 2 * A.ax.s + 2
    N = torch.empty((A.ngp, L), dtype=F64, device=A.device)
    dN = torch.empty_like(N)
    first = torch.empty(A.ngp, dtype=torch.int32, device=A.device)
    capi.taps_shape1d(h, A.basis, A.xg, N, dN, first)
    val = torch.empty((A.ngp, V.shape[1]), dtype=F64, device=A.device)
    der = torch.empty_like(val)
    capi.taps_interp1d(h, N, first, A.n, V, val)
    capi.taps_interp1d(h, dN, first, A.n, V, der)
    return val.T.contiguous(), der.T.contiguous()


def _loads(h, case, axes):
    X, Y, Z, T = axes
    one = lambda A, k=1: A.source(capi.SRC_POLY, [1.0]).expand(k, A.ngp)
    if case.source == "poly":
        L, a = case.axes[0].hi, case.amp
        mk, nk, mc, nc = case.m_k, case.n_k, case.m_c, case.n_c
        fx = torch.cat([X.source(capi.SRC_POLY, [0.0, 0.0, 2 * mc * a * a * L * L, -4 * mc * a * a * L,
                                                 2 * mc * a * a]),
                        X.source(capi.SRC_POLY, [0.0, nc * a * L, -nc * a]),
                        X.source(capi.SRC_POLY, [-mk * a * a * L * L, 6 * mk * a * a * L, -6 * mk * a * a]),
                        X.source(capi.SRC_POLY, [2 * nk * a])])
        ft = torch.cat([T.source(capi.SRC_POLY, [0.0, 1.0]), one(T), T.source(capi.SRC_POLY, [0.0, 0.0, 1.0]),
                        T.source(capi.SRC_POLY, [0.0, 1.0])])
        return [fx, one(Y, 4), one(Z, 4), ft], [None] * 4
    at = case.axes[3]
    amp = 2.0 * case.eta * case.power / (math.pi * case.radius ** 2 * case.axes[2].hi)
    centers = torch.tensor(case.x_start + case.speed * at.nodes(), dtype=F64, device=X.device)
    yc = torch.tensor([case.y0], dtype=F64, device=X.device)
    fx = X.source(capi.SRC_GAUSS, [amp, case.radius], n_cols=at.n, centers=centers)
    fy = Y.source(capi.SRC_GAUSS, [1.0, case.radius], n_cols=1, centers=yc)
    ft = T.source(capi.SRC_NODAL, [], n_cols=at.n)
    zero = np.zeros(at.n, dtype=np.int32)
    return [fx, fy, one(Z), ft], [np.arange(at.n), zero, zero, np.arange(at.n)]


def coefficient_problem(h, case, V, device="cuda"):
    """The linear problem of one global stage with the coefficients
    n + m u_c, u_c = prod_d V_d (V: device factors n_d x R_c, or None for
    the constant coefficients)."""
    Rc = 0 if V is None else int(V[0].shape[1])
    ax, ay, az, at = case.axes
    base = [[capi.MASS, capi.STIFF]] * 3 + [[capi.MASS, capi.DDT]]
    axes = []
    for d, A in enumerate(case.axes):
        weighted = [capi.WMASS, capi.WSTIFF if d < 3 else capi.WDDT]
        axes.append(DeviceAxis(h, A, base[d] + weighted * Rc, device))
    f_g, cols = _loads(h, case, axes)
    for d, A in enumerate(axes):
        # constant kinds and the loads, then each coefficient mode's weighted pair
        F = torch.empty((A.n, f_g[d].shape[0]), dtype=F64, device=device)
        capi.taps_assemble1d(h, A.basis, base[d], A.band[:2], f_g=f_g[d].contiguous(), F=F, n_loads=f_g[d].shape[0])
        A.F = F
        if Rc:
            val, der = _gauss_values(h, A, V[d])
            for r in range(Rc):
                coef = torch.cat([val[r], der[r]]).contiguous()
                capi.taps_assemble1d(h, A.basis, [capi.WMASS, capi.WSTIFF if d < 3 else capi.WDDT],
                                     A.band[2 + 2 * r: 4 + 2 * r], coef_g=coef)
    terms = [(case.n_c, (0, 0, 0, 1)), (case.n_k, (1, 0, 0, 0)), (case.n_k, (0, 1, 0, 0)), (case.n_k, (0, 0, 1, 0))]
    for r in range(Rc):
        w, k = 2 + 2 * r, 3 + 2 * r
        terms += [(case.m_c, (w, w, w, k)), (case.m_k, (k, w, w, w)), (case.m_k, (w, k, w, w)),
                  (case.m_k, (w, w, k, w))]
    return DeviceProblem(h, axes, terms, cols, case.M)


def compression_problem(h, prob, U, Rc):
    """Mode compression of u = prod_d U_d to R_c modes: operator M (x) M (x)
    M (x) M, loads M_d U_d (every fixed row of u kept fixed)."""

    class _View:
        def __init__(self, A, F):
            self.ax, self.n, self.kinds = A.ax, A.n, [capi.MASS]
            self.band, self.F, self.fixed, self.device = A.band[0:1], F, A.fixed, A.device

    views = []
    for A, u in zip(prob.axes, U):
        F = torch.empty_like(u)
        capi.taps_band_apply(h, A.ax.s, A.band[0], u, F)
        views.append(_View(A, F))
    return DeviceProblem(h, views, [(1.0, (0, 0, 0, 0))], [None] * 4, Rc)


def change(h, prob, V_new, V_old):
    """||u_c(new) - u_c(old)||_M / ||u_c(new)||_M through taps_td_inner."""
    s = [A.ax.s for A in prob.axes]
    bands = [A.band[0] for A in prob.axes]
    Rc = int(V_new[0].shape[1])
    out = torch.empty(3 * (Rc * Rc + 1), dtype=F64, device=V_new[0].device)
    k = Rc * Rc + 1
    capi.taps_td_inner(h, s, bands, V_new, V_new, out[0:k])
    capi.taps_td_inner(h, s, bands, V_old, V_old, out[k:2 * k])
    capi.taps_td_inner(h, s, bands, V_new, V_old, out[2 * k:3 * k])
    nn, oo, no = (float(v) for v in out[[k - 1, 2 * k - 1, 3 * k - 1]].cpu())
    return math.sqrt(max(nn + oo - 2.0 * no, 0.0) / nn) if nn > 0 else float("inf")


def global_local(h, case, U0, Rc, outer, sweeps, comp_sweeps=4, tol=0.0, V_init=None):
    """Algorithm 2.  U0: host or device initial factors of u; V_init: the
    compression's first initial factors (host, n_d x R_c).  Returns the
    device factors of u and of the compressed coefficient field, and the
    change per global stage (1.0 for the first)."""
    prob = coefficient_problem(h, case, None)
    U = prob.factors(U0) if isinstance(U0[0], np.ndarray) else [u.clone() for u in U0]
    V, changes = None, []
    for it in range(outer):
        if it:
            prob = coefficient_problem(h, case, V)
        capi.taps_als(h, prob.struct, U, 0.0, sweeps)                       # global stage
        comp = compression_problem(h, prob, U, Rc)                          # local stage
        Vn = comp.factors(V_init) if V is None else [v.clone() for v in V]
        capi.taps_als(h, comp.struct, Vn, 0.0, comp_sweeps)
        changes.append(1.0 if V is None else change(h, prob, Vn, V))
        V = Vn
        if tol > 0.0 and changes[-1] <= tol:
            break
    return U, V, changes
