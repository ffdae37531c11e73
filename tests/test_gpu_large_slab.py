"""The large single slab at its full size: x and y with 15000 nodes over
15 mm, z with 15 nodes, t with 513 nodes, M = 60 (fast diagonalisation with
the M <= 64 kernels), and the 2048^3 reconstruction around the melt pool.

The oracle cannot solve the 15000-row dim systems in a test's time (a plain
banded LU of 900k unknowns takes minutes), so parity here is on what it can
compute at this size and on properties that hold at any size:
  * the projected residual of the GPU's factors after two sweeps (oracle
    Grams, couplings and residual: every dim's rows);
  * each dim's couplings and force at those factors;
  * the dim solves: z and t against the oracle's solve (condition bar), x and
    y by their backward error in the oracle's arithmetic on every row;
  * the reconstruction: BF16 / FP32 planes against the oracle's FP64 values
    at sampled points within the elementwise rounding bound, and every
    plane's maximum of the 2048^3 reduction within the bound of the FP64
    reduction's maximum.
"""
import math
import time

import numpy as np
import pytest

import parity_util as pu
import taps_workloads as W
from oracle import problems, reconstruct, separated

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

ORDER = {"mass": 0, "stiff": 1, "ddt": 1}
U32, U16 = 2.0 ** -24, 2.0 ** -8


def _say(*a):
    print("[large]", *a, flush=True)


def _bound(prec, M):
    Mp = 32 * math.ceil(M / 32) if prec == "bf16" else 16 * math.ceil(M / 16)
    c = (1 + U32) ** 7 * ((1 + U16) ** 2 if prec == "bf16" else 1.0) - 1
    gam = Mp * U32 / (1 - Mp * U32)
    return c + gam * (1 + c)


@pytest.fixture(scope="module")
def large(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, problem
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    case = W.large_slab()
    _say(f"set-up {[a.n for a in case.axes]} M={case.M}")
    dev = problem.heat_slab(h, case)
    U = dev.factors(W.initial_factors(case.axes, case.M, case.seed))
    torch.cuda.synchronize()
    t = time.perf_counter()
    sweeps, rho, hist = capi.taps_als(h, dev.struct, U, 0.0, 2)
    torch.cuda.synchronize()
    _say(f"two sweeps in {time.perf_counter() - t:.2f} s (first includes workspace growth), rho {hist}")
    assert sweeps == 2 and np.isfinite(rho), capi.last_error(h)
    t = time.perf_counter()
    ora = problems.heat_slab(case)
    _say(f"oracle set-up {time.perf_counter() - t:.1f} s")
    yield torch, capi, h, case, dev, ora, U, rho
    capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)
    h.close()


def test_residual_of_the_sweeps(large):
    torch, capi, h, case, dev, ora, U, rho = large
    Uh = [u.cpu().numpy() for u in U]
    out = torch.empty(ora.D + 2, dtype=torch.float64, device="cuda")
    capi.taps_residual(h, dev.struct, U, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    Rs, Qs = separated.residuals(ora, Uh)
    ro = separated.residual_norm(ora, Uh)
    for d in range(ora.D):
        # the last-solved dim's residual is rounding noise of its own solve:
        # compared at the rounding scale of its force, not relative to itself
        ref, qd = float(np.sum(Rs[d] ** 2)), float(np.sum(Qs[d] ** 2))
        _say(f"dim {d}: ||R||/||Q|| gpu {np.sqrt(o[d] / qd):.3e} oracle {np.sqrt(ref / qd):.3e}")
        assert abs(o[d] - ref) <= pu.TOL * ref + (1e4 * pu.EPS) ** 2 * qd, (d, o[d], ref, qd)
    _say(f"rho gpu {o[-1]:.12e} (Algorithm 1's last {rho:.12e}) oracle {ro:.12e}")
    assert abs(o[-1] - ro) <= pu.TOL * ro
    assert abs(rho - ro) <= pu.TOL * ro


def test_contractions_and_dim_solves(large):
    torch, capi, h, case, dev, ora, U, rho = large
    M = case.M
    Uh = [u.cpu().numpy() for u in U]
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    berr = torch.zeros(1, dtype=torch.float64, device="cuda")
    for d in range(ora.D):
        n = ora.n[d]
        Cd = torch.empty((2, M, M), dtype=torch.float64, device="cuda")
        Qd = torch.empty((n, M), dtype=torch.float64, device="cuda")
        capi.taps_contract(h, dev.struct, d, 0xFF, U, Cd, Qd)
        Xd = torch.empty_like(Qd)
        capi.taps_solve_dim(h, dev.struct, d, Cd, Qd, Xd, info, berr)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        Co = separated.couplings(ora, Uh, d)
        Qo = separated.force(ora, Uh, d)
        for nm, c in Co.items():
            pu.check(Cd[ORDER[nm]].cpu().numpy(), c, pu.TOL, f"C dim {d} {nm}")
        pu.check(Qd.cpu().numpy(), Qo, pu.TOL, f"Q dim {d}")
        X = Xd.cpu().numpy()
        free = np.ones(n, bool)
        free[list(ora.fixed[d])] = False
        R = (separated.apply_dim(ora, d, Co, X) - Qo)[free]
        back = pu.rel(R + Qo[free], Qo[free])
        # normwise backward error (residual over ||operator|| ||X|| + ||Q||, the
        # operator's norm bounded by sum_k ||A^k||_F ||C^k||_F): a fast-
        # diagonalisation solve is backward stable up to the condition of the
        # eigenvector matrix P of E = C2^T C1^-T (the oracle's couplings)
        opn = sum(float(np.sqrt(ora.mats[d][k].multiply(ora.mats[d][k]).sum())) * np.linalg.norm(Ck)
                  for k, Ck in Co.items())
        eta = float(np.linalg.norm(R) / (opn * np.linalg.norm(X) + np.linalg.norm(Qo[free])))
        C1, C2 = Co["mass"], Co["stiff" if "stiff" in Co else "ddt"]
        E = C2.T @ np.linalg.inv(C1.T)
        condP = float(np.linalg.cond(np.linalg.eig(E)[1]))
        back_bar = max(1e-13, 100 * condP * pu.EPS)
        msg = (f"dim {d} (n={n}): normwise backward error {eta:.2e} (bar {back_bar:.1e}, cond(P) {condP:.1e}); "
               f"||R|| / ||Q|| {back:.2e} (the library's own {float(berr.item()):.2e})")
        if n <= 1000:
            Xo = separated.solve_dim(ora, d, Co, Qo)
            kappa = pu.cond_estimate(ora, d, Co)
            bar = max(pu.TOL, 10 * kappa * pu.EPS)
            r, m = pu.check(X, Xo, bar, f"X dim {d}")
            msg += f"; against the oracle's solve rel {r:.2e} max entry {m:.2e} (kappa {kappa:.1e}, bar {bar:.1e})"
        _say(msg)
        assert eta <= back_bar
        assert back < 1e-9          # far below the library's breakdown limit (1e-8)
        assert np.all(X[~free] == 0.0)


def _axis_points(lo, hi, n):
    return lo + (hi - lo) * (np.arange(n) + 0.5) / n


def test_subvolume_reconstruction(large):
    """2048^3 points around the melt pool at the slab's end time (x and y
    2.048 mm wide about the beam's last position, z over the whole depth):
    BF16 and FP32 against the FP64 oracle."""
    torch, capi, h, case, dev, ora, U, rho = large
    M, n = case.M, 2048
    xe = case.x_start + case.speed * case.axes[3].hi
    pts = [_axis_points(xe - 1.024, xe + 1.024, n), _axis_points(case.y0 - 1.024, case.y0 + 1.024, n),
           _axis_points(0.0, case.axes[2].hi, n)]
    Phis = []
    for d, p in enumerate(pts):
        L = 2 * case.axes[d].s + 2
        N = torch.empty((n, L), dtype=torch.float64, device="cuda")
        first = torch.empty(n, dtype=torch.int32, device="cuda")
        dp = torch.tensor(p, device="cuda")
        capi.taps_shape1d(h, dev.axes[d].basis, dp, N, None, first)
        P = torch.empty((n, M), dtype=torch.float64, device="cuda")
        capi.taps_interp1d(h, N, first, case.axes[d].n, U[d], P)
        Phis.append(P)
    w = U[3][-1].contiguous()                     # time factor at t = T_s as mode weights
    torch.cuda.synchronize()
    Ph = [P.cpu().numpy() for P in Phis]
    wh = w.cpu().numpy()
    red = {}
    for prec in ("fp64", "fp32", "bf16"):
        out = torch.full((n, 4), float("nan"), dtype=torch.float64, device="cuda")
        p = {"fp64": capi.FP64, "fp32": capi.FP32, "bf16": capi.BF16}[prec]
        torch.cuda.synchronize()
        t = time.perf_counter()
        capi.taps_reconstruct(h, Phis, M, out, prec=p, mode=capi.REDUCE, mode_w=w, thr=100.0)
        torch.cuda.synchronize()
        red[prec] = out.cpu().numpy()
        _say(f"2048^3 {prec} reduction in {1e3 * (time.perf_counter() - t):.1f} ms; "
             f"hottest plane max {red[prec][:, 0].max():.4f} K")
    # per plane: the largest term-magnitude sum over the plane bounds every
    # point's rounding error, hence the error of the plane's maximum
    amax = [np.abs(P).max(axis=0) for P in Ph[:2]]
    Tk = (np.abs(Ph[2]) * np.abs(wh)[None, :]) @ (amax[0] * amax[1])
    for prec in ("fp32", "bf16"):
        err = np.abs(red[prec][:, 0] - red["fp64"][:, 0])
        assert np.all(err <= _bound(prec, M) * Tk), prec
        _say(f"  {prec} plane maxima: worst |err| / term bound {np.max(err / (_bound(prec, M) * Tk)):.2e}, "
             f"worst |err| {err.max():.2e} K")
    # sampled points of a few planes (the top surface, where the pool is)
    rng = np.random.Generator(np.random.PCG64(3))
    ks = [n - 1, n // 2, 0]
    idx = np.concatenate([np.stack([rng.integers(0, n, 4000), rng.integers(0, n, 4000), np.full(4000, k)], -1)
                          for k in ks])
    ref = reconstruct.reconstruct_points(Ph, idx, wh)
    T = reconstruct.abs_term_sum(Ph, idx, wh)
    for prec in ("fp32", "bf16"):
        p = {"fp32": capi.FP32, "bf16": capi.BF16}[prec]
        sub = [Phis[0], Phis[1], Phis[2][ks].contiguous()]
        out = torch.empty((len(ks), n, n), dtype=torch.float32, device="cuda")
        capi.taps_reconstruct(h, sub, M, out, prec=p, mode=capi.STORE, mode_w=w)
        torch.cuda.synchronize()
        g = out.cpu().numpy()
        kk = np.repeat(np.arange(len(ks)), 4000)
        got = g[kk, idx[:, 0], idx[:, 1]].astype(np.float64)
        ratio = np.abs(got - ref) / np.maximum(T, 1e-300)
        _say(f"  {prec} sampled points: worst |err| / sum|terms| {ratio.max():.2e} (bound {_bound(prec, M):.2e}), "
             f"rel L2 {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
        assert ratio.max() <= _bound(prec, M)
    # the FP64 reduction's top-plane maximum is that of the oracle's values
    # on that plane's sampled points at most
    assert red["fp64"][n - 1, 0] >= ref[:4000].max() - 1e-9 * max(1.0, abs(ref[:4000].max()))
