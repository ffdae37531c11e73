"""Space-time slab chain with a carried initial condition and mode compression
(driver above the C ABI; every numeric step runs in the library's kernels).

Paper, LPBF section (split u = u_c + u_0 with a homogeneous initial condition
for u_0) and the mode-compression appendix.  For slab T+1:

  * the carried field u_c = sum_r V_x[:,r] V_y[:,r] V_z[:,r] is constant in
    time, so it enters the slab equation as 3 K_c extra separable load terms
    -k (A_x V_x) (A_y V_y) (A_z V_z) w_t, with the stiffness matrix in one
    spatial dim and the mass matrix in the other two, and w_t = int Ntilde dt;
  * after Algorithm 1, u(x, t_max) = u_c + sum_m U_x U_y U_z U_t[n_t-1, m]
    (K_c + M modes) is compressed to K_c modes by Algorithm 1 on the
    mass-only operator with the loads M_d W_d.

Loads are formed with taps_band_apply (banded 1D matrix times factor columns),
the slab and the compression are solved with taps_als.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import capi
from .problem import F64, DeviceAxis, DeviceProblem


class _AxisView:
    """A dimension of the compression problem: one kind (mass) of a slab axis."""

    def __init__(self, axis: DeviceAxis, F):
        self.ax = axis.ax
        self.n = axis.n
        self.kinds = [capi.MASS]
        self.band = axis.band[0:1]          # MASS is kind 0 of every slab axis
        self.F = F
        self.fixed = axis.fixed
        self.device = axis.device


def slab_problem(h, case, V=None, device="cuda", M=None):
    """Device heat slab of ``case`` (moving source) plus the carried field
    V = [V_x, V_y, V_z] (device, n_d x K_c; None for the first slab)."""
    M = case.M if M is None else M
    ax, ay, az, at = case.axes
    Kc = 0 if V is None else V[0].shape[1]
    nc = 3 * Kc
    # grid-only data shared by every slab on the grid (the loads are per slab,
    # apart from the time loads, which depend on the grid and K_c alone)
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device, shared=True)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device, shared=True)
    Z = DeviceAxis(h, az, [capi.MASS, capi.STIFF], device, shared=True)
    T = DeviceAxis(h, at, [capi.MASS, capi.DDT], device, shared=True)
    pad = lambda A, f: torch.cat([f, torch.zeros((nc, A.ngp), dtype=F64, device=device)]) if nc else f
    amp = 2.0 * case.eta * case.power / (math.pi * case.radius ** 2 * case.depth)
    centers = torch.tensor(case.x_start + case.speed * at.nodes(), dtype=F64, device=device)
    yc = torch.tensor([case.y0], dtype=F64, device=device)
    X.assemble(pad(X, X.source(capi.SRC_GAUSS, [amp, case.radius], n_cols=at.n, centers=centers)))
    Y.assemble(pad(Y, Y.source(capi.SRC_GAUSS, [1.0, case.radius], n_cols=1, centers=yc)))
    Z.assemble(pad(Z, Z.source(capi.SRC_TOPLAYER, [case.height, case.depth])))
    def time_loads():
        ft = T.source(capi.SRC_NODAL, [], n_cols=at.n)
        return torch.cat([ft, T.source(capi.SRC_POLY, [1.0])]) if Kc else ft   # w_t = int Ntilde dt

    T.assemble_shared(("nodal", bool(Kc)), time_loads)
    nt = at.n
    if Kc:
        # carried terms j = 0, 1, 2 (stiffness in spatial dim j), column j*Kc + r
        for e, A in enumerate((X, Y, Z)):
            r0 = A.F.shape[1] - nc
            for j in range(3):
                kind = 1 if e == j else 0
                alpha = -case.k if e == 0 else 1.0
                capi.taps_band_apply(h, A.ax.s, A.band[kind], V[e], A.F[:, r0 + j * Kc: r0 + (j + 1) * Kc],
                                     alpha=alpha)
    rc, k = case.rho_cp_per_ms, case.k
    terms = [(rc, (0, 0, 0, 1)), (k, (1, 0, 0, 0)), (k, (0, 1, 0, 0)), (k, (0, 0, 1, 0))]
    extra = np.arange(nc, dtype=np.int32)
    cols = [np.concatenate([np.arange(nt), nt + extra]).astype(np.int32),
            np.concatenate([np.zeros(nt), 1 + extra]).astype(np.int32),
            np.concatenate([np.zeros(nt), 1 + extra]).astype(np.int32),
            np.concatenate([np.arange(nt), np.full(nc, nt)]).astype(np.int32)]
    prob = DeviceProblem(h, [X, Y, Z, T], terms, cols, M)
    prob.keep += [centers, yc]
    return prob


def compression_problem(h, slab: DeviceProblem, V, U, Kc: int):
    """Mode compression of u(x, t_max) = u_c + sum_m prod U_d U_t[n_t-1]:
    operator M (x) M (x) M, loads M_d W_d with W = [V | U diag(U_t[-1]) in x]."""
    kin = 0 if V is None else V[0].shape[1]
    M = U[0].shape[1]
    views = []
    for e in range(3):
        A = slab.axes[e]
        F = torch.empty((A.n, kin + M), dtype=F64, device=A.device)
        if kin:
            capi.taps_band_apply(h, A.ax.s, A.band[0], V[e], F[:, :kin])
        capi.taps_band_apply(h, A.ax.s, A.band[0], U[e], F[:, kin:], scale=U[3][-1] if e == 0 else None)
        views.append(_AxisView(A, F))
    return DeviceProblem(h, views, [(1.0, (0, 0, 0))], [None] * 3, Kc)


def run_chain(h, cases, U0s, C0s, sweeps: int, comp_sweeps: int, V0=None, device="cuda"):
    """Slabs in order with a carried K_c-mode field (K_c = mode count of C0s[T]).

    U0s[T], C0s[T]: host initial factors of slab T and of its compression;
    each slab runs ``sweeps`` and each compression ``comp_sweeps`` sweeps of
    Algorithm 1.  Returns per slab (U, V_in, V_out) as device tensors."""
    out = []
    V = V0
    for T, case in enumerate(cases):
        prob = slab_problem(h, case, V, device)
        U = prob.factors(U0s[T])
        capi.taps_als(h, prob.struct, U, 0.0, sweeps)
        cprob = compression_problem(h, prob, V, U, C0s[T][0].shape[1])
        Vn = cprob.factors(C0s[T])
        capi.taps_als(h, cprob.struct, Vn, 0.0, comp_sweeps)
        out.append((U, V, Vn))
        V = Vn
    return out
