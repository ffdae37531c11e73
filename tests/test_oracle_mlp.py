"""Pins of the warm-start network oracle: BF16 rounding against a brute-force
nearest search, GELU and the layer gradients against central differences,
the first Adam step against its closed form."""
import numpy as np

from oracle import mlp


def test_bf16_round_known_values():
    u = 2.0 ** -7                                     # BF16 spacing on [1, 2)
    cases = {1.0: 1.0, 1 + u / 2: 1.0, 1 + 1.5 * u: 1 + 2 * u, 1 + u / 2 + 2 ** -20: 1 + u,
             -(1 + 1.5 * u): -(1 + 2 * u), 0.0: 0.0, 3.0: 3.0}
    for x, want in cases.items():
        assert mlp.bf16_round(np.array([x]))[0] == want, x
    assert np.isinf(mlp.bf16_round(np.array([np.inf]))[0])


def test_bf16_round_is_nearest_with_ties_to_even():
    rng = np.random.Generator(np.random.PCG64(0))
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 6, 20000)).astype(np.float32).astype(np.float64)
    got = mlp.bf16_round(x)
    e = np.floor(np.log2(np.abs(x)))
    ulp = 2.0 ** (e - 7)
    lo = np.floor(x / ulp) * ulp
    hi = lo + ulp
    dlo, dhi = x - lo, hi - x
    even_lo = (np.round(lo / ulp) % 2) == 0
    want = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(even_lo, lo, hi)))
    assert np.array_equal(got, want)


def test_gelu_derivative():
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(z)).max() < 1e-8
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-12


def test_backward_matches_central_differences():
    widths = [5, 7, 6, 4]
    Ws, bs = mlp.init(widths, 1)
    rng = np.random.Generator(np.random.PCG64(2))
    for b in bs:
        b += 0.1 * rng.standard_normal(b.shape)
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 4))
    Y, cache = mlp.forward(Ws, bs, X)
    L, dY = mlp.loss(Y, T)
    dWs, dbs = mlp.backward(Ws, bs, cache, dY)
    h = 1e-6
    for l in range(3):
        for (i, j) in [(0, 0), (1, 2), (widths[l + 1] - 1, widths[l] - 1)]:
            Wp = [w.copy() for w in Ws]; Wp[l][i, j] += h
            Wm = [w.copy() for w in Ws]; Wm[l][i, j] -= h
            fd = (mlp.loss(mlp.forward(Wp, bs, X)[0], T)[0] - mlp.loss(mlp.forward(Wm, bs, X)[0], T)[0]) / (2 * h)
            assert abs(fd - dWs[l][i, j]) <= 1e-7 * max(1.0, abs(fd)), (l, i, j)
        bp = [b.copy() for b in bs]; bp[l][0] += h
        bm = [b.copy() for b in bs]; bm[l][0] -= h
        fd = (mlp.loss(mlp.forward(Ws, bp, X)[0], T)[0] - mlp.loss(mlp.forward(Ws, bm, X)[0], T)[0]) / (2 * h)
        assert abs(fd - dbs[l][0]) <= 1e-7 * max(1.0, abs(fd))


def test_bf16_mode_rounds_inputs_and_weights():
    widths = [4, 3, 2]
    Ws, bs = mlp.init(widths, 3)
    X = np.random.Generator(np.random.PCG64(4)).standard_normal((5, 4))
    Y, cache = mlp.forward(Ws, bs, X, mode="bf16")
    # same as the FP64 network on rounded weights, with the input of each layer rounded
    a = X
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = mlp.bf16_round(a) @ mlp.bf16_round(W).T + b
        a = mlp.gelu(z) if l < 1 else z
    assert np.array_equal(Y, a)


def test_first_adam_step_closed_form():
    g = np.array([0.3, -2.0, 1e-9, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    opt = mlp.Adam([p], lr=0.01)
    opt.step([p], [g])
    want = 1.0 - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, want, rtol=0, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.Generator(np.random.PCG64(5))
    X = rng.uniform(-1, 1, (64, 3))
    T = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], X[:, 2] ** 2], axis=1)
    Ws, bs = mlp.init([3, 32, 32, 2], 6)
    opt = mlp.Adam(Ws + bs, lr=3e-3)
    first = None
    for it in range(1500):
        Y, cache = mlp.forward(Ws, bs, X)
        L, dY = mlp.loss(Y, T)
        first = L if first is None else first
        dWs, dbs = mlp.backward(Ws, bs, cache, dY)
        opt.step(Ws + bs, dWs + dbs)
    assert L < first / 50
