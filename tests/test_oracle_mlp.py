"""Pin the float64 predictor reference: finite differences and closed forms."""
import numpy as np
import pytest

from oracle import mlp
from paper_2508_16376_amd import workloads as W


def _params(seed, bias_scale=0.1):
    p = W.mlp_init_weights(seed).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    r = (W.counter_values(seed + 1, 0, 64 + 64 + 1) >> np.uint64(11)).astype(np.float64) / (1 << 53)
    return mlp.pack(W1, (r[:64] - 0.5) * bias_scale, W2, (r[64:128] - 0.5) * bias_scale, W3, r[128] - 0.5)


def _batch(seed, B=16):
    r = (W.counter_values(seed, 0, B * 7) >> np.uint64(11)).astype(np.float64) / (1 << 53)
    x = (r[:B * 6].reshape(B, 6) - 0.5) * 4
    y = r[B * 6:] * 10
    return x, y


def _away_from_kinks(p, x, margin=1e-3):
    _, (x, z1, h1, z2, h2) = mlp.forward(p, x)
    return np.abs(z1).min() > margin and np.abs(z2).min() > margin


def test_parameter_count():
    assert mlp.N_PARAMS == 4673
    assert W.mlp_init_weights(1).size == 4673


@pytest.mark.parametrize("seed", [3, 17, 29])
def test_gradient_matches_central_differences(seed):
    p = _params(seed)
    x, y = _batch(seed + 100)
    # pick a batch that keeps every pre-activation away from the ReLU kink
    for k in range(50):
        if _away_from_kinks(p, x):
            break
        x, y = _batch(seed + 200 + k)
    assert _away_from_kinks(p, x)
    L, g = mlp.grad(p, x, y)
    assert abs(L - mlp.loss(p, x, y)) < 1e-12
    idx = np.unique(np.concatenate([np.arange(0, mlp.N_PARAMS, 23), np.arange(mlp.N_PARAMS - 70, mlp.N_PARAMS)]))
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (mlp.loss(pp, x, y) - mlp.loss(pm, x, y)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (i, fd, g[i])


def test_dead_second_layer_closed_form():
    """W2 = 0: h2 = relu(b2) for every sample, the first layer gets no gradient,
    and out = W3 . relu(b2) + b3."""
    p = _params(5)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    b2 = np.abs(b2) + 0.1
    p = mlp.pack(W1, b1, np.zeros_like(W2), b2, W3, b3)
    x, y = _batch(7, 32)
    out, _ = mlp.forward(p, x)
    np.testing.assert_allclose(out, np.full(32, W3 @ b2 + b3), rtol=1e-12)
    L, g = mlp.grad(p, x, y)
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unpack(g)
    assert np.all(gW1 == 0) and np.all(gb1 == 0)
    r = out - y
    np.testing.assert_allclose(gb3, 2 * r.mean(), rtol=1e-12)
    np.testing.assert_allclose(gW3, 2 * r.mean() * b2, rtol=1e-12)
    # every second-layer unit is active (b2 > 0), so dW2 = outer(W3, sum_s d_out_s h1_s)
    h1 = np.maximum(x @ W1.T + b1, 0)
    np.testing.assert_allclose(gW2, np.outer(W3, (2 * r / 32) @ h1), rtol=1e-10, atol=1e-14)


def test_linear_region_matches_matrix_product():
    """With every unit active the network is the affine map W3 W2 (W1 x + b1) + W3 b2 + b3."""
    p = _params(9)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    W1, W2 = np.abs(W1) * 0.1, np.abs(W2) * 0.1
    b1, b2 = np.abs(b1) + 5, np.abs(b2) + 5
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    x, y = _batch(11, 20)
    x = np.abs(x)
    out, _ = mlp.forward(p, x)
    A = W3 @ W2 @ W1
    c = W3 @ (W2 @ b1 + b2) + b3
    np.testing.assert_allclose(out, x @ A + c, rtol=1e-12)
    L, g = mlp.grad(p, x, y)
    r = out - y
    gW1 = mlp.unpack(g)[0]
    # d/dW1 of mean (x A + c - y)^2 where A = W3 W2 W1: outer(W2^T W3, sum_s 2 r_s x_s / B)
    np.testing.assert_allclose(gW1, np.outer(W2.T @ W3, (2 * r / 20) @ x), rtol=1e-10)


def test_first_adam_step_is_sign_step():
    """After one step with bias correction, m_hat = g and v_hat = g^2, so the
    update is -lr * g / (|g| + eps)."""
    p = _params(13)
    x, y = _batch(15, 8)
    _, g = mlp.grad(p, x, y)
    z = np.zeros_like(p)
    p1, m, v = mlp.adam_step(p, g, z, z, 1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)


def test_training_reduces_loss_on_a_learnable_target():
    x, _ = _batch(21, 512)
    y = 2.0 * x[:, 0] - x[:, 3] + 0.5
    p = _params(23)
    p2, losses = mlp.train(p, x, y, epochs=30, batch=64, lr=3e-3)
    assert losses[-1] < 0.05 * losses[0]
