"""Pins of the CPU reference network (oracle/mlp.py)."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-8, 8, 5000), [0.0, 1.0, -2.5, 3.0e-5]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_gradient_against_finite_differences():
    """Exact FP64 network (no BF16 rounding): analytic gradient = central differences."""
    rng = np.random.default_rng(1)
    w = rng.standard_normal(mlp.NW) * 0.3
    X = rng.standard_normal((37, mlp.IN))
    Y = rng.standard_normal(37)
    loss, g = mlp.loss_and_grad(w, X, Y, bf=False)
    h = 1e-6
    idx = rng.choice(mlp.NW, 60, replace=False).tolist() + [mlp.O_B3, mlp.O_W3, mlp.O_B1 + 3, mlp.O_W2 + 70]
    for k in idx:
        wp = w.copy(); wp[k] += h
        wm = w.copy(); wm[k] -= h
        fd = (mlp.loss_and_grad(wp, X, Y, bf=False)[0] - mlp.loss_and_grad(wm, X, Y, bf=False)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_forward_matches_plain_matmul():
    rng = np.random.default_rng(2)
    w = rng.standard_normal(mlp.NW)
    X = rng.standard_normal((5, mlp.IN))
    W1, b1, W2, b2, w3, b3 = mlp.unpack(w)
    ref = np.maximum(np.maximum(X @ W1.T + b1, 0) @ W2.T + b2, 0) @ w3 + b3
    assert np.allclose(mlp.forward(w, X, bf=False)[0], ref, rtol=1e-13)
