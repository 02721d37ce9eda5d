"""Pins for the FP64 cost-model reference: finite differences of the loss,
hand-computed forward values, Adam's first step, and bfloat16 rounding."""

import numpy as np

from oracle import mlp


def test_layout_size():
    assert mlp.TOTAL == 4553 and mlp.TRAINABLE == 4545


def test_forward_by_hand():
    d = {k: np.zeros(s) if s else 0.0 for k, (o, s) in mlp.OFFSETS.items()}
    d["sigma"] = np.ones(4)
    d["b3"] = 0.25
    p = mlp.pack(d)
    assert np.allclose(mlp.forward(p, np.ones((3, 4))), 0.25)
    # one live path: h1_0 = relu(x0 - 1), h2_0 = 2*h1_0, y = 3*h2_0 - 1
    d["W1"][0, 0] = 1.0
    d["b1"][0] = -1.0
    d["W2"][0, 0] = 2.0
    d["w3"][0] = 3.0
    d["b3"] = -1.0
    p = mlp.pack(d)
    X = np.array([[0.5, 0, 0, 0], [3.0, 9, 9, 9]])
    assert np.allclose(mlp.forward(p, X), [-1.0, 3 * 2 * 2.0 - 1.0])
    # standardisation
    d["mu"] = np.array([1.0, 0, 0, 0])
    d["sigma"] = np.array([2.0, 1, 1, 1])
    p = mlp.pack(d)
    assert np.allclose(mlp.forward(p, np.array([[7.0, 0, 0, 0]])), [3 * 2 * 2.0 - 1.0])


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init(3)
    p[mlp.OFFSETS["mu"][0]:mlp.OFFSETS["mu"][0] + 4] = [0.1, -0.2, 0.3, 0.0]
    p[mlp.OFFSETS["sigma"][0]:mlp.OFFSETS["sigma"][0] + 4] = [1.5, 0.7, 1.0, 2.0]
    X = rng.normal(size=(37, 4))
    t = rng.normal(size=37)
    g = mlp.grad(p, X, t)
    idx = rng.choice(mlp.TRAINABLE, 200, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])
    assert not g[mlp.TRAINABLE:].any()


def test_adam_first_step_is_signed_lr():
    p = mlp.init(1)
    g = np.zeros(mlp.TOTAL)
    sign = np.where(np.arange(mlp.TRAINABLE) % 2 == 0, 1.0, -1.0)
    g[:mlp.TRAINABLE] = sign * np.linspace(0.01, 1, mlp.TRAINABLE)
    p2, m, v = mlp.adam(p, np.zeros(mlp.TOTAL), np.zeros(mlp.TOTAL), g, 0.01, 1)
    # bias-corrected first step of Adam moves every weight by lr * sign(g) (up to eps)
    assert np.allclose(p2[:mlp.TRAINABLE] - p[:mlp.TRAINABLE], -0.01 * np.sign(g[:mlp.TRAINABLE]), atol=1e-7)


def test_bfloat16_round_to_nearest_even():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.1415927, 65504.0, 0.0], np.float32)
    want = [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 3.140625, 65536.0, 0.0]
    assert np.array_equal(mlp.bf16(vals), want)
    assert np.isnan(mlp.bf16(np.array([np.nan], np.float32)))[0]


def test_spearman():
    assert abs(mlp.spearman(np.arange(10), np.arange(10) ** 3) - 1) < 1e-12
    assert abs(mlp.spearman(np.arange(10), -np.arange(10)) + 1) < 1e-12


def test_forward_bf16_by_hand():
    # One live path, with a value chosen to round at each of the points where
    # the BF16 inference rounds (weights, standardised input, each hidden
    # activation; mu and sigma stay FP32; the output accumulates exactly).
    d = {k: np.zeros(s) if s else 0.0 for k, (o, s) in mlp.OFFSETS.items()}
    d["mu"] = np.array([0.5, 0, 0, 0])
    d["sigma"] = np.array([0.5, 1, 1, 1])
    d["W1"][0, 0] = 1 + 2 ** -8          # bf16: a tie, rounds to even -> 1.0
    d["W2"][0, 0] = 1 + 2 ** -7          # exact in bf16
    d["w3"][0] = 2.0
    d["b3"] = 0.5
    p = mlp.pack(d)
    # x = 1.005859375: (x - 0.5) / 0.5 = 1.01171875 = 1 + 3*2^-8 -> bf16 rounds up to 1 + 2^-6
    x = np.array([[1.005859375, 0, 0, 0]])
    xs = 1 + 2 ** -6
    h1 = 1.0 * xs                         # 1.015625, exact in bf16
    a2 = (1 + 2 ** -7) * h1               # 1.0235595703125 -> bf16 1.0234375 (spacing 2^-7)
    h2 = 1.0234375
    assert a2 == 1.0235595703125
    want = 2.0 * h2 + 0.5                 # 2.546875
    assert mlp.forward_bf16(p, x)[0] == want == 2.546875
    # the FP32/FP64 path keeps every digit and so differs
    exact = 2.0 * ((1 + 2 ** -7) * ((1 + 2 ** -8) * 1.01171875)) + 0.5
    assert abs(mlp.forward(p, x)[0] - exact) < 1e-12 and mlp.forward(p, x)[0] != want
    # a negative pre-activation is cut by the ReLU before rounding
    x2 = np.array([[0.25, 0, 0, 0]])      # xs = -0.5 -> h1 = 0 -> y = b3
    assert mlp.forward_bf16(p, x2)[0] == 0.5
