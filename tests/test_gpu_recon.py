"""Reduced-precision reconstruction on the matrix cores against the FP64 oracle.

The field is u[i][j][k] = sum_m w_m Phi_0[i,m] Phi_1[j,m] Phi_2[k,m] (paper
Sec. 2.3, TD interpolation).  The GPU's BF16 and FP32 paths round at fixed
points (factors to FP32, s = w*Phi_2, a' = Phi_0*s, then BF16 operands for the
BF16 path) and accumulate in FP32; the elementwise bound below follows from
those rounding points and the standard bound for recursive summation:

    |u_gpu - u| <= (c + gamma_Mp (1 + c)) * sum_m |w_m Phi_0 Phi_1 Phi_2|,
    c = (1+u32)^7 (1+u16)^2 - 1  (BF16),   c = (1+u32)^7 - 1  (FP32),
    gamma_Mp = Mp u32 / (1 - Mp u32),  u32 = 2^-24, u16 = 2^-8,

with Mp the mode count padded to the MFMA inner size (zero modes add nothing).
Every element is checked against it; the measured worst ratio is printed.
"""
import math

import numpy as np
import pytest

from oracle import reconstruct

pytestmark = pytest.mark.gpu

U32, U16 = 2.0 ** -24, 2.0 ** -8


def bound(prec, M):
    Mp = 32 * math.ceil(M / 32) if prec == "bf16" else 16 * math.ceil(M / 16)
    c = (1 + U32) ** 7 * ((1 + U16) ** 2 if prec == "bf16" else 1.0) - 1
    gam = Mp * U32 / (1 - Mp * U32)
    return c + gam * (1 + c)


def _say(*a):
    print("[recon]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi
    h = capi.Handle()
    yield torch, capi, h
    h.close()


def factors(shape, M, seed):
    """Random factors with decaying mode scales, like converged TAPS modes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Phis = [rng.standard_normal((n, M)) for n in shape]
    w = rng.standard_normal(M) * np.exp(-0.15 * np.arange(M))
    return Phis, w


def run(env, Phis, w, prec, mode, thr=0.0):
    torch, capi, h = env
    n0, n1, n2 = (P.shape[0] for P in Phis)
    M = Phis[0].shape[1]
    dP = [torch.tensor(P, device="cuda") for P in Phis]
    dw = torch.tensor(w, device="cuda")
    p = capi.BF16 if prec == "bf16" else capi.FP32
    if mode == "store":
        out = torch.full((n2, n0, n1), float("nan"), dtype=torch.float32, device="cuda")
        capi.taps_reconstruct(h, dP, M, out, prec=p, mode=capi.STORE, mode_w=dw)
    else:
        out = torch.full((n2, 4), float("nan"), dtype=torch.float64, device="cuda")
        capi.taps_reconstruct(h, dP, M, out, prec=p, mode=capi.REDUCE, mode_w=dw, thr=thr)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


CASES = [  # (n0, n1, n2, M): ragged row blocks and column tiles, all paddings
    (300, 77, 5, 40),
    (17, 33, 3, 13),
    (257, 16, 2, 64),
    (5, 3, 4, 1),
    (1, 1, 1, 7),
    (512, 130, 2, 33),
    (1030, 64, 2, 60),
]


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
@pytest.mark.parametrize("shape_M", CASES, ids=lambda c: "x".join(map(str, c)))
def test_store_within_bound(env, prec, shape_M):
    n0, n1, n2, M = shape_M
    _say(f"store {prec} {n0}x{n1}x{n2} M={M}")
    Phis, w = factors((n0, n1, n2), M, seed=n0 + 7 * M)
    got = run(env, Phis, w, prec, "store").transpose(1, 2, 0)   # -> [i][j][k]
    assert np.all(np.isfinite(got))
    ref = reconstruct.reconstruct_grid(Phis, w)
    idx = np.stack(np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij"), -1).reshape(-1, 3)
    T = reconstruct.abs_term_sum(Phis, idx, w).reshape(n0, n1, n2)
    ratio = np.abs(got - ref) / np.maximum(T, 1e-300)
    b = bound(prec, M)
    _say(f"  worst |err|/sum|terms| = {ratio.max():.3e} (bound {b:.3e}), rel L2 = "
         f"{np.linalg.norm(got - ref) / np.linalg.norm(ref):.3e}")
    assert ratio.max() <= b


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_reduce_consistent_with_fp64(env, prec):
    n0, n1, n2, M = 300, 77, 5, 40
    _say(f"reduce {prec} {n0}x{n1}x{n2} M={M}")
    Phis, w = factors((n0, n1, n2), M, seed=11)
    ref = reconstruct.reconstruct_grid(Phis, w)
    thr = float(np.quantile(ref, 0.9))
    r = run(env, Phis, w, prec, "reduce", thr=thr)
    idx = np.stack(np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij"), -1).reshape(-1, 3)
    e = bound(prec, M) * reconstruct.abs_term_sum(Phis, idx, w).reshape(n0, n1, n2)
    for k in range(n2):
        u, ek = ref[:, :, k], e[:, :, k]
        assert u.max() - ek.max() <= r[k, 0] <= u.max() + ek.max()
        # sum of squares: per-point error plus FP32 partial sums of 16 values
        ss_tol = np.sum(2 * np.abs(u) * ek + ek ** 2) + 16 * U32 * 1.01 * np.sum((np.abs(u) + ek) ** 2)
        assert abs(r[k, 1] - np.sum(u ** 2)) <= ss_tol
        # count of u > thr lies between the counts with the threshold moved by the bound
        assert np.sum(u - ek > thr) <= r[k, 2] <= np.sum(u + ek > thr)
        assert r[k, 3] == 0.0


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_large_plane_sampled(env, prec):
    """2048 x 2048 planes with M = 60 (the large-slab reconstruction shape) on
    sampled points, plus the reduction of the same planes."""
    n0, n1, n2, M = 2048, 2048, 3, 60
    _say(f"large {prec} {n0}x{n1}x{n2} M={M}")
    Phis, w = factors((n0, n1, n2), M, seed=5)
    got = run(env, Phis, w, prec, "store")                      # [k][i][j]
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.stack([rng.integers(0, n, 20000) for n in (n0, n1, n2)], -1)
    idx = np.concatenate([idx, [[0, 0, 0], [n0 - 1, n1 - 1, n2 - 1], [n0 - 1, 0, 1], [0, n1 - 1, 2]]])
    ref = reconstruct.reconstruct_points(Phis, idx, w)
    T = reconstruct.abs_term_sum(Phis, idx, w)
    g = got[idx[:, 2], idx[:, 0], idx[:, 1]]
    ratio = np.abs(g - ref) / T
    _say(f"  worst sampled |err|/sum|terms| = {ratio.max():.3e} (bound {bound(prec, M):.3e})")
    assert ratio.max() <= bound(prec, M)
    # thresholds that most of the plane exceeds, and that only its hottest
    # points exceed (most tiles then hold no point above it): the reduction
    # of the same products gives the stored plane's maximum and count exactly
    hot = float(np.float32(np.quantile(got, 0.9995)))
    for thr in (0.0, hot):
        r = run(env, Phis, w, prec, "reduce", thr=thr)
        for k in range(n2):
            plane = got[k]
            assert r[k, 0] == plane.max()
            assert r[k, 2] == np.sum(plane > thr)
            assert abs(r[k, 1] - np.sum(plane.astype(np.float64) ** 2)) <= 1e-5 * np.sum(plane.astype(np.float64) ** 2)
        _say(f"  thr {thr:.4g}: counts {[int(c) for c in r[:, 2]]} equal the stored planes'")


def test_reduced_precision_rejects_oversized_plane(env):
    torch, capi, h = env
    _say("oversized plane rejected")
    P = [torch.zeros((n, 4), dtype=torch.float64, device="cuda") for n in (1 << 16, 1 << 15, 1)]
    out = torch.empty((1, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        capi.taps_reconstruct(h, P, 4, out, prec=capi.BF16, mode=capi.REDUCE)


@pytest.mark.parametrize("prec,mode", [("bf16", "reduce"), ("bf16", "store"), ("fp32", "reduce"), ("fp64", "reduce")])
def test_batched_fields_equal_single_calls(env, prec, mode):
    # several fields of one shape in one call: each output bit-identical to
    # its own single-field call (ragged plane sizes, one field without weights)
    torch, capi, h = env
    shape, M, B = (70, 45, 9), 40, 5
    P = {"bf16": capi.BF16, "fp32": capi.FP32, "fp64": capi.FP64}[prec]
    md = capi.REDUCE if mode == "reduce" else capi.STORE
    dt = torch.float64 if (md == capi.REDUCE or P == capi.FP64) else torch.float32
    size = (shape[2], 4) if md == capi.REDUCE else (shape[0] * shape[1] * shape[2],)
    fields, ws, outs, refs = [], [], [], []
    for b in range(B):
        Phis, w = factors(shape, M, 100 + b)
        fields.append([torch.tensor(Q, device="cuda") for Q in Phis])
        ws.append(None if b == 2 else torch.tensor(w, device="cuda"))
        outs.append(torch.full(size, float("nan"), dtype=dt, device="cuda"))
        refs.append(torch.full(size, float("nan"), dtype=dt, device="cuda"))
    _say(f"batched {prec} {mode}: {B} fields {shape} M={M}")
    capi.taps_reconstruct_batched(h, fields, M, outs, prec=P, mode=md, mode_ws=ws, thr=0.5)
    for b in range(B):
        capi.taps_reconstruct(h, fields[b], M, refs[b], prec=P, mode=md, mode_w=ws[b], thr=0.5)
    torch.cuda.synchronize()
    for b in range(B):
        assert torch.equal(outs[b], refs[b]), b
