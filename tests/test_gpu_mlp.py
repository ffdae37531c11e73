"""Warm-start kernels against the oracle: network forward and backward layer
by layer (on the device's own cached BF16 inputs, so only FP32 summation
separates the two), squared-error loss, Adam, canonical factor form, coarse
sampling/prolongation and initial-condition features."""
import numpy as np
import pytest

import taps_workloads as W
from oracle import mlp, warmstart as ows

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _say(*a):
    print("[mlp]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, warmstart
    h = capi.Handle()
    yield torch, capi, warmstart, h
    h.close()


def read_cache(cache, widths, B):
    """Split the activation cache (layout documented with taps_mlp_cache_bytes)."""
    raw = cache.cpu().numpy()
    off, xs, zs = 0, [], []
    a256 = lambda n: (n + 255) // 256 * 256
    for l in range(len(widths) - 1):
        ld = (widths[l] + 31) // 32 * 32
        xb = raw[off: off + B * ld * 2].view(np.uint16).reshape(B, ld)
        xs.append((xb.astype(np.uint32) << 16).view(np.float32).astype(np.float64))
        off += a256(B * ld * 2)
        zs.append(raw[off: off + B * widths[l + 1] * 4].view(np.float32).reshape(B, widths[l + 1]).astype(np.float64))
        off += a256(B * widths[l + 1] * 4)
    return xs, zs


def dev_weights(net):
    """Device BF16 weights as float64 (unpadded)."""
    out = []
    for l, Q in enumerate(net.w16):
        q = Q.cpu().numpy().view(np.uint16)[:, : net.widths[l]]
        out.append((q.astype(np.uint32) << 16).view(np.float32).astype(np.float64))
    return out


WIDTHS = [67, 256, 256, 256, 96]


def build(env, B, seed=0):
    torch, capi, ws, h = env
    Ws, bs = W.mlp_init(WIDTHS, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    bs = [0.1 * rng.standard_normal(b.shape) for b in bs]
    net = ws.Net(h, WIDTHS, Ws, bs)
    X = rng.standard_normal((B, WIDTHS[0])).astype(np.float32)
    return net, X, [np.asarray(b, np.float32).astype(np.float64) for b in bs], Ws


def test_weights_rounded_to_bf16(env):
    torch, capi, ws, h = env
    net, X, bs, Ws = build(env, 5)
    for l, Wd in enumerate(dev_weights(net)):
        assert np.array_equal(Wd, mlp.bf16_round(np.asarray(Ws[l], np.float32)))
        pad = net.w16[l].cpu().numpy()[:, WIDTHS[l]:]
        assert np.all(pad == 0)


@pytest.mark.parametrize("B", [1, 37, 128])
def test_forward_layerwise(env, B):
    torch, capi, ws, h = env
    _say(f"forward B={B}")
    net, X, bs, _ = build(env, B)
    Y = net.forward(torch.tensor(X, device="cuda")).cpu().numpy().astype(np.float64)
    xs, zs = read_cache(net.cache(B), WIDTHS, B)
    Wd = dev_weights(net)
    assert np.array_equal(xs[0][:, :67], mlp.bf16_round(X)) and np.all(xs[0][:, 67:] == 0)
    for l in range(len(WIDTHS) - 1):
        inp = WIDTHS[l]
        ref = xs[l][:, :inp] @ Wd[l].T + bs[l]
        bound = (inp + 2) * U32 * (np.abs(xs[l][:, :inp]) @ np.abs(Wd[l]).T + np.abs(bs[l])) + 1e-30
        assert np.all(np.abs(zs[l] - ref) <= bound), l
        if l < len(WIDTHS) - 2:
            want = mlp.bf16_round(mlp.gelu(zs[l]))
            got = xs[l + 1][:, : WIDTHS[l + 1]]
            diff = got != want
            # FP32 GELU may round across a BF16 boundary: rare, and then by one BF16 step
            assert diff.mean() < 0.01
            ulp = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(want), 1e-30))) - 7)
            assert np.all(np.abs(got - want)[diff] <= 1.01 * ulp[diff])
    assert np.array_equal(Y, zs[-1])


def test_backward_layerwise(env):
    torch, capi, ws, h = env
    B = 37
    _say("backward B=37")
    net, X, bs, _ = build(env, B, seed=3)
    net.forward(torch.tensor(X, device="cuda"))
    dY = np.random.Generator(np.random.PCG64(4)).standard_normal((B, WIDTHS[-1])).astype(np.float32)
    net.backward(B, torch.tensor(dY, device="cuda"))
    torch.cuda.synchronize()
    xs, zs = read_cache(net.cache(B), WIDTHS, B)
    Wd = dev_weights(net)
    L = len(WIDTHS) - 1
    g = dY.astype(np.float64)
    for l in reversed(range(L)):
        inp = WIDTHS[l]
        dz = g * mlp.gelu_grad(zs[l]) if l < L - 1 else g
        gW = dz.T @ xs[l][:, :inp]
        gb = dz.sum(axis=0)
        got = net.grads[l].cpu().numpy().astype(np.float64)
        gotb = net.grads[L + l].cpu().numpy().astype(np.float64)
        e = np.linalg.norm(got[:, :inp] - gW) / np.linalg.norm(gW)
        eb = np.linalg.norm(gotb - gb) / np.linalg.norm(gb)
        _say(f"  layer {l}: dW rel {e:.2e}, db rel {eb:.2e}")
        assert e < 2e-5 and eb < 2e-5
        assert np.all(got[:, inp:] == 0)
        g = dz @ Wd[l]


def test_mse_and_adam(env):
    torch, capi, ws, h = env
    rng = np.random.Generator(np.random.PCG64(7))
    Y = rng.standard_normal(1000).astype(np.float32)
    T = rng.standard_normal(1000).astype(np.float32)
    dY = torch.empty(1000, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    capi.taps_mlp_mse(h, torch.tensor(Y, device="cuda"), torch.tensor(T, device="cuda"), dY, loss)
    L, dref = mlp.loss(Y.astype(np.float64), T.astype(np.float64))
    assert abs(loss.item() - L) <= 1e-12 * L
    assert np.abs(dY.cpu().numpy() - dref).max() <= 2 * U32 * np.abs(dref).max()
    p0 = rng.standard_normal(500)
    p = torch.tensor(p0.astype(np.float32), device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    ref = [p0.astype(np.float32).astype(np.float64)]
    opt = mlp.Adam(ref, lr=1e-2)
    for t in range(1, 6):
        gr = rng.standard_normal(500).astype(np.float32)
        capi.taps_adam_step(h, p, torch.tensor(gr, device="cuda"), m, v, 1e-2, t)
        opt.step(ref, [gr.astype(np.float64)])
    assert np.abs(p.cpu().numpy() - ref[0]).max() <= 1e-5


def test_canonicalize_matches_oracle(env):
    torch, capi, ws, h = env
    rng = np.random.Generator(np.random.PCG64(8))
    U = [rng.standard_normal((n, 9)) for n in (40, 33, 17, 25)]
    U[2][:, 4] = 0.0                                    # a mode with a zero column
    dU = [torch.tensor(u, device="cuda") for u in U]
    out = [torch.empty_like(u) for u in dU]
    capi.taps_canonicalize(h, dU, out)
    ref = ows.canonicalize(U)
    for o, r in zip(out, ref):
        assert np.abs(o.cpu().numpy() - r).max() <= 1e-13 * max(1.0, np.abs(r).max())


def test_coarse_sampling_prolongation_and_ic_features(env):
    torch, capi, ws, h = env
    case = W.heat_slab(40, 48, 16, 33, M=3)
    ax = case.axes[1]
    rng = np.random.Generator(np.random.PCG64(9))
    U = rng.standard_normal((ax.n, 5))
    c = ws.Coarse(h, ax, 32)
    dU = torch.tensor(U, device="cuda")
    Uc = c.sample(dU)
    assert np.abs(Uc.cpu().numpy() - ows.sample(ax, U, 32)).max() < 1e-12
    Uf = c.prolong(Uc)
    assert np.abs(Uf.cpu().numpy() - ows.prolong(ax, Uc.cpu().numpy())).max() < 1e-12
    V = [rng.standard_normal((a.n, 3)) for a in case.axes[:3]]
    V[2][0, :] = 0.0
    c4 = [ws.Coarse(h, a, 4) for a in case.axes[:3]]
    f = ws.ic_features(h, c4, [torch.tensor(v, device="cuda") for v in V]).cpu().numpy()
    assert np.abs(f - ows.ic_features(case.axes, V)).max() < 1e-12
