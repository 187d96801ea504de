"""Pins for the seeder's FP64 MLP oracle: central finite differences of the
loss; Adam (Kingma & Ba 2015) at step 1 in closed form, over many steps of a
constant gradient (geometric moment sums) and over three steps of changing
gradients with moments worked out by hand; the min-over-seeds argmin on
hand-made cases; bfloat16 rounding against torch's conversion; and the
bfloat16 emulation of the backward pass: equal to the exact pass on data that
is already bfloat16, rounding locations on a hand-computed 1-1-1 net, and
within the bfloat16 error of the exact pass on a random net."""
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


def test_adam_constant_gradient_every_step():
    """Constant gradient g: the moments are geometric sums, m_t = (1 - b1^t) g
    and v_t = (1 - b2^t) g^2, so the bias-corrected moments are g and g^2 at
    every step and each step moves a parameter by -lr g / (|g| + eps)."""
    params = small_net()
    grads = [(rng.normal(size=W.shape) + 0.1, rng.normal(size=b.shape) - 0.1) for W, b in params]
    opt = mlp.Adam(params, lr=1e-3)
    cur = params
    for t in range(1, 13):
        new = opt.step(cur, grads)
        for i, ((W, b), (Wn, bn), (gW, gb)) in enumerate(zip(cur, new, grads)):
            for j, (p, pn, g) in enumerate(((W, Wn, gW), (b, bn, gb))):
                np.testing.assert_allclose(opt.m[i][j], (1 - 0.9 ** t) * g, rtol=1e-12)
                np.testing.assert_allclose(opt.v[i][j], (1 - 0.999 ** t) * g * g, rtol=1e-12)
                np.testing.assert_allclose(pn - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-7)
        cur = new
    assert opt.t == 12


def test_adam_varying_gradient_hand_values():
    """Three steps with changing gradients; the moments after each step and
    the bias-correction factors are written out by hand from the recursions
    m_t = 0.9 m + 0.1 g, v_t = 0.999 v + 0.001 g^2 (zero start), and the
    steps follow -lr (m_t / c1_t) / (sqrt(v_t / c2_t) + eps)."""
    W0 = np.array([[0.5, -0.25, 2.0]])
    b0 = np.array([1.0])
    gs = [np.array([[1.0, 0.0, 4.0]]), np.array([[-2.0, 3.0, 4.0]]), np.array([[0.5, 0.0, -4.0]])]
    m_hand = [[0.1, 0.0, 0.4], [-0.11, 0.3, 0.76], [-0.049, 0.27, 0.284]]
    v_hand = [[0.001, 0.0, 0.016], [0.004999, 0.009, 0.031984], [0.005244001, 0.008991, 0.047952016]]
    c1_hand = [0.1, 0.19, 0.271]
    c2_hand = [0.001, 0.001999, 0.002997001]
    opt = mlp.Adam([(W0, b0)], lr=1e-3)
    cur = [(W0, b0)]
    for t in range(3):
        new = opt.step(cur, [(gs[t], np.zeros(1))])
        m, v = np.array(m_hand[t]), np.array(v_hand[t])
        np.testing.assert_allclose(opt.m[0][0][0], m, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(opt.v[0][0][0], v, rtol=1e-12, atol=1e-15)
        step = -1e-3 * (m / c1_hand[t]) / (np.sqrt(v / c2_hand[t]) + 1e-8)
        np.testing.assert_allclose(new[0][0][0] - cur[0][0][0], step, rtol=1e-9, atol=1e-15)
        # a zero gradient with zero moments leaves the bias where it is
        assert new[0][1][0] == b0[0]
        cur = new


def test_bf16_backward_equals_exact_on_bf16_exact_data():
    """Where every value the emulation rounds is already a bfloat16 number,
    the emulated gradients equal the exact (finite-difference-pinned) ones:
    a linear layer on bfloat16 weights, inputs and upstream gradients; and a
    two-layer net whose hidden pre-activations are all 0 (SiLU(0) = 0,
    SiLU'(0) = 1/2) with one-hot power-of-two upstream gradients."""
    W = mlp.bf16(rng.normal(size=(14, 7)))
    b = mlp.bf16(rng.normal(size=14))
    x = mlp.bf16(rng.normal(size=(9, 7)))
    dy = mlp.bf16(rng.normal(size=(9, 14)))
    for emu in (False, True):
        y, cache = mlp.forward([(W, b)], x, emulate_bf16=emu)
        g = mlp.backward([(W, b)], cache, dy, emulate_bf16=emu)
        if not emu:
            ref = g
    np.testing.assert_array_equal(g[0][0], ref[0][0])
    np.testing.assert_array_equal(g[0][1], ref[0][1])
    W1, b1 = np.zeros((5, 7)), np.zeros(5)
    W2, b2 = mlp.bf16(rng.normal(size=(14, 5))), mlp.bf16(rng.normal(size=14))
    dy = np.zeros((9, 14))
    dy[np.arange(9), rng.integers(0, 14, size=9)] = 2.0 ** rng.integers(-4, 4, size=9)
    outs = []
    for emu in (False, True):
        y, cache = mlp.forward([(W1, b1), (W2, b2)], x, emulate_bf16=emu)
        outs.append(mlp.backward([(W1, b1), (W2, b2)], cache, dy, emulate_bf16=emu))
    for (a, c) in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a[0], c[0])
        np.testing.assert_array_equal(a[1], c[1])
    assert np.abs(outs[1][0][0]).max() > 0          # the first layer's dW is exercised


def test_bf16_rounding_locations_hand_computed():
    """A 1 -> 1 -> 1 net (x = 1, both weights 1, biases 0) where the rounding
    points matter, with values worked out by hand.  SiLU(1) = 0.7310585786...
    rounds to 187/256 = 0.73046875 in bfloat16 (spacing 2^-8 on [0.5, 1));
    SiLU'(1) = 0.9276705... rounds to 237/256 = 0.92578125.  The emulation
    rounds the stored activation (forward output, dW of layer 2) and the
    upstream gradient that multiplies the inputs (dW of layer 1), but not the
    gradient summed into the bias.  With dy = 1/3 (bfloat16 342/1024 =
    0.333984375, spacing 2^-9 on [0.25, 0.5)) the layer-1 gradient
    0.333984375 * SiLU'(1) = 0.3098... rounds to 159/512 = 0.310546875."""
    import math
    params = [(np.array([[1.0]]), np.array([0.0])), (np.array([[1.0]]), np.array([0.0]))]
    x = np.array([[1.0]])
    sig = 1.0 / (1.0 + math.exp(-1.0))
    silu1, dsilu1 = sig, sig * (1.0 + (1.0 - sig))
    y, cache = mlp.forward(params, x, emulate_bf16=True)
    assert y[0, 0] == 0.73046875
    g = mlp.backward(params, cache, np.array([[1.0]]), emulate_bf16=True)
    assert g[1][0][0, 0] == 0.73046875 and g[1][1][0] == 1.0
    assert g[0][0][0, 0] == 0.92578125
    assert g[0][1][0] == pytest.approx(dsilu1, rel=1e-15)
    g = mlp.backward(params, cache, np.array([[1.0 / 3.0]]), emulate_bf16=True)
    assert g[1][0][0, 0] == 0.333984375 * 0.73046875
    assert g[1][1][0] == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert g[0][0][0, 0] == 0.310546875
    assert g[0][1][0] == pytest.approx(0.333984375 * dsilu1, rel=1e-15)
    # exact mode keeps every value
    y, cache = mlp.forward(params, x)
    g = mlp.backward(params, cache, np.array([[1.0]]))
    assert y[0, 0] == pytest.approx(silu1, rel=1e-15)
    assert g[1][0][0, 0] == pytest.approx(silu1, rel=1e-15)
    assert g[0][0][0, 0] == pytest.approx(dsilu1, rel=1e-15)


def test_bf16_backward_close_to_exact():
    """On a random 4-layer net the emulated gradients stay within the
    bfloat16 error (a few 2^-8 relative per tensor) of the exact ones, and
    differ from them (the rounding is applied)."""
    params = small_net((7, 64, 64, 64, 56))
    x = rng.normal(size=(32, 7))
    q = rng.normal(size=(32, 7))
    ge, gx = [], []
    for emu, dst in ((True, ge), (False, gx)):
        y, cache = mlp.forward(params, x, emulate_bf16=emu)
        _, _, dy = mlp.min_over_k_loss(y, q, 8)
        dst.extend(mlp.backward(params, cache, dy, emulate_bf16=emu))
    for (a, c) in zip(ge, gx):
        for u, v in zip(a, c):
            rel = np.linalg.norm(u - v) / np.linalg.norm(v)
            assert 0 < rel < 3e-2
