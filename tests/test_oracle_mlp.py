"""Pins for the seeder's FP64 MLP oracle: central finite differences of the
loss, Adam's first step in closed form (Kingma & Ba 2015: the bias-corrected
first step is -lr * g / (|g| + eps)), the min-over-seeds argmin on hand-made
cases, and bfloat16 rounding against torch's conversion."""
import numpy as np
import pytest

from oracle import mlp

rng = np.random.default_rng(11)


def small_net(sizes=(7, 16, 16, 16, 14)):
    import synth
    return synth.mlp_init(list(sizes), 3)


def loss_of(params, x, q, K):
    y, _ = mlp.forward(params, x)
    return mlp.min_over_k_loss(y, q, K)[0]


def test_gradients_match_finite_differences():
    params = small_net()
    K = 2
    x = rng.normal(size=(5, 7))
    q = rng.normal(size=(5, 7))
    y, cache = mlp.forward(params, x)
    _, _, dy = mlp.min_over_k_loss(y, q, K)
    grads = mlp.backward(params, cache, dy)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for (arr, g) in ((W, grads[li][0]), (b, grads[li][1])):
            idx = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]
            for ix in idx:
                old = arr[ix]
                arr[ix] = old + h
                lp = loss_of(params, x, q, K)
                arr[ix] = old - h
                lm = loss_of(params, x, q, K)
                arr[ix] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[ix]) <= 1e-6 * max(1.0, abs(fd)), (li, ix, fd, g[ix])


def test_adam_first_step_closed_form():
    params = small_net()
    grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in params]
    opt = mlp.Adam(params, lr=1e-3)
    new = opt.step(params, grads)
    for (W, b), (Wn, bn), (gW, gb) in zip(params, new, grads):
        np.testing.assert_allclose(Wn - W, -1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-9)
        np.testing.assert_allclose(bn - b, -1e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-9)


def test_min_over_k_argmin_and_ties():
    q = np.zeros((3, 7))
    y = np.zeros((3, 21))
    y[0, :7] = 1.0          # sample 0: seeds (1, 0.5, 0.2) -> k = 2
    y[0, 7:14] = 0.5
    y[0, 14:] = 0.2
    y[1, :7] = 0.3          # sample 1: tie between k = 0 and k = 2 -> 0
    y[1, 7:14] = 0.9
    y[1, 14:] = -0.3
    y[2, 7:14] = 0.0        # sample 2: k = 1 exact
    y[2, :7] = 2.0
    y[2, 14:] = 1.0
    loss, k, g = mlp.min_over_k_loss(y, q, 3)
    np.testing.assert_array_equal(k, [2, 0, 1])
    assert loss == pytest.approx((7 * 0.04 + 7 * 0.09 + 0.0) / 3)
    # gradient only on the winning seed
    assert np.all(g[0, :14] == 0) and np.all(g[1, 7:] == 0) and np.all(g[2, :7] == 0)
    np.testing.assert_allclose(g[0, 14:], 2 * 0.2 / 3)


def test_bf16_rounding_matches_torch():
    import torch
    x = np.concatenate([rng.normal(size=1000) * 10 ** rng.uniform(-8, 8, size=1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)


def test_bf16_forward_close_to_exact():
    params = small_net((7, 64, 64, 64, 56))
    x = rng.normal(size=(32, 7))
    y, _ = mlp.forward(params, x)
    yb, _ = mlp.forward(params, x, emulate_bf16=True)
    assert np.linalg.norm(yb - y) / np.linalg.norm(y) < 2e-2


def test_encode_targets():
    p = np.array([[0.3, 0.0, 0.4]])
    qt = np.array([[-0.5, 0.5, 0.5, 0.5]])
    x = mlp.encode_targets(p, qt, reach=0.5)
    np.testing.assert_allclose(x, [[0.6, 0.0, 0.8, 0.5, -0.5, -0.5, -0.5]])
