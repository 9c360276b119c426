"""Pins of the surrogate network's CPU reference (oracle/mlp.py) against what does not
depend on it: the parameter count the configuration states, an independent bfloat16
conversion (PyTorch's), finite differences of the loss, and Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def _theta(seed=0, scale=0.3):
    return np.random.default_rng(seed).normal(0.0, scale, mlp.N_PARAMS)


def test_parameter_count_and_layout():
    assert mlp.N_PARAMS == 8770
    th = np.arange(mlp.N_PARAMS, dtype=np.float64)
    layers = mlp.unpack(th)
    assert [W.shape for W, _ in layers] == [(4, 64), (64, 64), (64, 64), (64, 2)]
    assert layers[0][1][0] == 256 and layers[3][1][-1] == mlp.N_PARAMS - 1


def test_bf16_rounding_matches_an_independent_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 3, 20000), rng.uniform(-1e-3, 1e-3, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_gradient_is_the_derivative_of_the_loss():
    rng = np.random.default_rng(2)
    x, t = rng.normal(size=(13, 4)), rng.normal(size=(13, 2))
    w = rng.uniform(0.2, 1.0, 13)
    th = _theta(3)
    L, g = mlp.loss_and_grad(th, x, t, w, mixed=False)
    h = 1e-6
    for i in list(range(0, 320, 37)) + list(range(320, mlp.N_PARAMS, 611)) + [mlp.N_PARAMS - 1]:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, x, t, w, mixed=False)[0] -
              mlp.loss_and_grad(tm, x, t, w, mixed=False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_mixed_precision_gradient_stays_near_fp64():
    rng = np.random.default_rng(4)
    x, t = rng.normal(size=(64, 4)), rng.normal(size=(64, 2))
    th = _theta(5)
    _, g64 = mlp.loss_and_grad(th, x, t, mixed=False)
    _, g16 = mlp.loss_and_grad(th, x, t, mixed=True)
    assert np.linalg.norm(g16 - g64) / np.linalg.norm(g64) < 2e-2


def test_adam_first_step_moves_each_weight_by_the_learning_rate():
    rng = np.random.default_rng(6)
    th, g = _theta(7), rng.normal(size=mlp.N_PARAMS)
    z = np.zeros(mlp.N_PARAMS)
    new, m, v = mlp.adam(th, g, z, z, 1, 1e-3)
    assert np.allclose(new - th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
