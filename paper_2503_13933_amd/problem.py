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


class DeviceAxis:
    """Nodes, basis descriptor, Gauss rule and bands of one dimension."""

    def __init__(self, h, ax, kinds, device):
        self.ax = ax
        self.n = ax.n
        self.x = torch.tensor(ax.nodes(), dtype=F64, device=device)
        self.basis = Basis1D(ax.n, self.x.data_ptr(), ax.s, float(ax.a), ax.p, ax.n_gauss)
        self.ngp = (ax.n - 1) * ax.n_gauss
        self.xg = torch.empty(self.ngp, dtype=F64, device=device)
        self.wg = torch.empty(self.ngp, dtype=F64, device=device)
        capi.taps_gauss_points(h, self.basis, self.xg, self.wg)
        self.kinds = list(kinds)
        self.band = torch.empty((len(kinds), ax.n, 4 * ax.s + 3), dtype=F64, device=device)
        self.fixed = torch.zeros(ax.n, dtype=torch.uint8, device=device)
        if ax.fixed:
            self.fixed[list(ax.fixed)] = 1
        self.F = None
        self.h = h
        self.device = device

    def source(self, kind, params, n_cols=1, centers=None):
        """Source factor(s) at the Gauss points, (n_cols, ngp)."""
        out = torch.empty((n_cols, self.ngp), dtype=F64, device=self.device)
        basis = self.basis if kind == capi.SRC_NODAL else None
        capi.taps_source1d(self.h, kind, self.xg, n_cols, params, out, centers=centers, basis=basis)
        return out

    def assemble(self, f_g):
        """Bands of self.kinds and load columns of f_g ((R, ngp) at the Gauss points)."""
        f_g = f_g.contiguous()
        R = f_g.shape[0]
        self.F = torch.empty((self.n, R), dtype=F64, device=self.device)
        capi.taps_assemble1d(self.h, self.basis, self.kinds, self.band, f_g=f_g, F=self.F, n_loads=R)
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
    X = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], device)
    Y = DeviceAxis(h, ay, [capi.MASS, capi.STIFF], device)
    Z = DeviceAxis(h, az, [capi.MASS, capi.STIFF], device)
    T = DeviceAxis(h, at, [capi.MASS, capi.DDT], device)
    amp = 2.0 * case.eta * case.power / (math.pi * case.radius ** 2 * case.depth)
    centers = torch.tensor(case.x_start + case.speed * at.nodes(), dtype=F64, device=device)
    X.assemble(X.source(capi.SRC_GAUSS, [amp, case.radius], n_cols=at.n, centers=centers))
    yc = torch.tensor([case.y0], dtype=F64, device=device)
    Y.assemble(Y.source(capi.SRC_GAUSS, [1.0, case.radius], n_cols=1, centers=yc))
    Z.assemble(Z.source(capi.SRC_TOPLAYER, [case.height, case.depth]))
    T.assemble(T.source(capi.SRC_NODAL, [], n_cols=at.n))
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


def build(h, case, device="cuda", M=None):
    if case.kind == "heat_slab":
        return heat_slab(h, case, device, M)
    if case.kind == "poisson2d":
        return poisson2d(h, case, device, M)
    raise ValueError(case.kind)
