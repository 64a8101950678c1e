"""Pins for the MLP oracle: BF16 rounding against torch's conversion and hand
values, a hand-computed forward pass, gradients against central finite
differences, Adam's closed form for the first step.  CPU only."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_hand_values():
    # 1 + 2^-8 is half way between 1 and 1 + 2^-7: ties to even -> 1
    assert mlp.bf16_round(1.0 + 2 ** -8) == 1.0
    # 1 + 3*2^-8 is half way between 1 + 2^-7 (odd mantissa) and 1 + 2^-6 (even)
    assert mlp.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert mlp.bf16_round(-2.0) == -2.0
    assert mlp.bf16_round(0.0) == 0.0


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.uniform(-1e-3, 1e-3, 5000)]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)


def _sparse_params(K):
    p = np.zeros(mlp.param_count(K))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, K)   # views into p
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0
    W3[0, :] = np.arange(K)
    b3[:] = 0.5
    return p


def test_forward_hand_example():
    K = 5
    p = _sparse_params(K)
    X = np.zeros((2, 16))
    X[0, 0] = 2.0      # passes both ReLUs: y_j = 2 j + 0.5
    X[1, 0] = -3.0     # blocked by the first ReLU: y_j = 0.5
    y, _ = mlp.forward(p, X, K)
    assert np.allclose(y[0], 2 * np.arange(K) + 0.5)
    assert np.allclose(y[1], 0.5)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    K, B = 7, 9
    p = mlp.bf16_round(rng.normal(0, 0.3, mlp.param_count(K)))
    X = rng.normal(0, 1, (B, 16))
    T = rng.normal(0, 1, (B, K))
    loss, g = mlp.loss_and_grads(p, X, T, K)
    idx = rng.choice(p.size, 60, replace=False)
    fd = mlp.finite_difference(p, X, T, K, idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-8)
    # the loss is the mean squared error of the forward pass
    y, _ = mlp.forward(p, X, K)
    assert abs(loss - np.mean((y - T) ** 2)) < 1e-12


def test_adam_first_step_closed_form():
    """After one Adam step from zero moments, the update is -lr*sign(g)
    (up to eps), whatever beta1 and beta2 are."""
    g = np.array([0.3, -2.0, 1e-3, -5e-2])
    w = np.zeros(4)
    w1 = mlp.adam_step(w, g, np.zeros(4), np.zeros(4), lr=0.01, b1=0.8, b2=0.95, eps=1e-12, step=1)[0]
    assert np.allclose(w1, -0.01 * np.sign(g))
