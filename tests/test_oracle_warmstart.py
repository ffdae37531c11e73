"""Pins of the warm-start data oracle: canonical form against a hand-worked
case and its invariants, coarse sampling/prolongation against polynomial
reproduction and the Kronecker-delta property, input features against a
separable field known in closed form."""
import numpy as np

import taps_workloads as W
from oracle import fulltensor, warmstart


def test_canonicalize_hand_worked():
    # mode 0: lambda = 1*1*1 = 1; mode 1: lambda = 2*... larger -> comes first
    U0 = np.array([[1.0, 2.0], [0.0, 0.0]])
    U1 = np.array([[0.0, 0.0], [1.0, -3.0]])        # mode 1 column norm 3, largest entry negative
    U2 = np.array([[-1.0, 0.5], [0.0, 0.0]])        # mode 0 column sign flips
    out = warmstart.canonicalize([U0, U1, U2])
    # mode 1 first: lambda = 2 * 3 * 0.5 = 3 > 1; its y column -> [0, 1] with scale -3, z -> [1, 0] scale 0.5
    assert np.allclose(out[0][:, 0], [2.0 * -3.0 * 0.5, 0.0])
    assert np.allclose(out[1][:, 0], [0.0, 1.0]) and np.allclose(out[2][:, 0], [1.0, 0.0])
    # mode 0 second: y [0,1] (norm 1, positive), z [-1, 0] -> sign -1
    assert np.allclose(out[0][:, 1], [-1.0, 0.0])
    assert np.allclose(out[1][:, 1], [0.0, 1.0]) and np.allclose(out[2][:, 1], [1.0, 0.0])


def test_canonicalize_invariants():
    rng = np.random.Generator(np.random.PCG64(0))
    U = [rng.standard_normal((n, 6)) for n in (7, 5, 4, 6)]
    out = warmstart.canonicalize(U)
    assert np.abs(fulltensor.td_tensor(out) - fulltensor.td_tensor(U)).max() < 1e-12
    lam = np.prod([np.linalg.norm(o, axis=0) for o in out], axis=0)
    assert np.all(np.diff(lam) <= 1e-12)
    for d in range(1, 4):
        assert np.allclose(np.linalg.norm(out[d], axis=0), 1.0)
        i = np.argmax(np.abs(out[d]), axis=0)
        assert np.all(out[d][i, np.arange(6)] > 0)
    # idempotent
    again = warmstart.canonicalize(out)
    assert all(np.allclose(a, b) for a, b in zip(again, out))


def test_zero_column_mode_left_unscaled():
    U = [np.array([[1.0, 2.0]]), np.array([[0.0, 3.0], [0.0, 4.0]])]
    out = warmstart.canonicalize(U)
    assert np.allclose(out[1][:, 0], [0.6, 0.8]) and np.allclose(out[0][:, 0], [10.0])
    assert np.allclose(out[1][:, 1], [0.0, 0.0]) and np.allclose(out[0][:, 1], [1.0])


def test_prolongation_reproduces_quadratics_and_sampling_inverts_it():
    ax = W.Axis("y", 0.0, 1.0, 48, 2, 20.0, 2, 5)
    x = ax.nodes()
    U = np.stack([1 + x, x * x - 0.3 * x, np.ones_like(x)], axis=1)
    Uc = warmstart.sample(ax, U, 32)
    xc = warmstart.coarse_nodes(ax, 32)
    assert np.allclose(Uc, np.stack([1 + xc, xc * xc - 0.3 * xc, np.ones_like(xc)], axis=1), atol=1e-12)
    Uf = warmstart.prolong(ax, Uc)
    assert np.abs(Uf - U).max() < 1e-12
    rng = np.random.Generator(np.random.PCG64(1))
    C = rng.standard_normal((32, 4))
    back = warmstart.sample(W.Axis("y", 0.0, 1.0, 32, 2, 20.0, 2, 5), C, 32)
    assert np.abs(back - C).max() < 1e-12


def test_ic_features_of_separable_field():
    case = W.heat_slab(20, 16, 9, 9, M=3, s=1, p=1)
    ax, ay, az = case.axes[:3]
    V = [ax.nodes()[:, None].copy(), np.ones((ay.n, 1)), az.nodes()[:, None].copy()]
    f = warmstart.ic_features(case.axes, V).reshape(4, 4, 4)
    xc, zc = warmstart.coarse_nodes(ax, 4), warmstart.coarse_nodes(az, 4)
    assert np.abs(f - xc[:, None, None] * zc[None, None, :]).max() < 1e-12
    assert np.all(warmstart.ic_features(case.axes, None) == 0.0)


def test_param_features_and_fallback_rule():
    lo = W.heat_slab(8, 8, 8, 8, power=100.0, radius=0.03, k=0.01, y0=0.3)
    hi = W.heat_slab(8, 8, 8, 8, power=300.0, radius=0.08, k=0.03, y0=0.7)
    assert np.allclose(warmstart.param_features(lo), -1.0) and np.allclose(warmstart.param_features(hi), 1.0)
    assert warmstart.restart_plain(2.0, 1.0, 1.5)          # worse than the plain median
    assert warmstart.restart_plain(1.0, 1.2, 1.5)          # grows from sweep 1 to 2
    assert not warmstart.restart_plain(1.0, 0.9, 1.5)
    # a breakdown (NaN residual) after either sweep is a loss, never a keep
    nan = float("nan")
    assert warmstart.restart_plain(nan, 0.9, 1.5)
    assert warmstart.restart_plain(1.0, nan, 1.5)
    assert warmstart.restart_plain(nan, nan, 1.5)
