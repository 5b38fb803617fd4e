"""Pins of the order-cost network's CPU reference (oracle/mlp.py).

Each test checks the reference against something other than itself: finite
differences, closed forms, the defining property of Adam's first step and
exactly representable bfloat16 values.
"""
import numpy as np

from oracle import mlp


def rand_net(rng, scale=0.3):
    return rng.normal(0.0, scale, mlp.N_WEIGHTS)


def test_weight_count_and_layout():
    assert mlp.N_WEIGHTS == 5825
    rng = np.random.default_rng(0)
    w = rand_net(rng)
    assert np.array_equal(mlp.pack(*mlp.unpack(w)), w)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    w = rand_net(rng)
    X = rng.normal(0.0, 1.0, (37, mlp.N_IN))
    T = rng.normal(0.0, 2.0, 37)
    loss, g = mlp.loss_and_grad(w, X, T)
    assert np.isclose(loss, np.mean((mlp.forward(w, X) - T) ** 2))
    # every bias and W3 weight, and a sample of W1 and W2 entries
    idx = list(range(24 * 64, 24 * 64 + 64)) + list(range(5825 - 129, 5825))
    idx += list(rng.choice(24 * 64, 60, replace=False))
    idx += list(24 * 64 + 64 + rng.choice(64 * 64, 60, replace=False))
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        lp, _ = mlp.loss_and_grad(wp, X, T)
        lm, _ = mlp.loss_and_grad(wm, X, T)
        num = (lp - lm) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)), (i, num, g[i])


def test_dead_hidden_layer_outputs_the_last_bias():
    # all first-layer pre-activations negative: y = relu(b2) . W3 + b3
    rng = np.random.default_rng(2)
    W1 = np.zeros((24, 64))
    b1 = -np.ones(64)
    W2 = rng.normal(size=(64, 64))
    b2 = rng.normal(size=64)
    W3 = rng.normal(size=64)
    b3 = 0.75
    w = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = rng.normal(size=(5, 24))
    expect = np.maximum(b2, 0.0) @ W3 + b3
    assert np.allclose(mlp.forward(w, X), expect)
    # gradient: only b2 (where positive), W3 and b3 move
    T = rng.normal(size=5)
    _, g = mlp.loss_and_grad(w, X, T)
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unpack(g)
    r = expect - T
    assert np.all(gW1 == 0) and np.all(gb1 == 0) and np.all(gW2 == 0)
    assert np.isclose(gb3, 2 * r.mean())
    assert np.allclose(gW3, 2 * r.mean() * np.maximum(b2, 0.0))
    assert np.allclose(gb2, 2 * r.mean() * W3 * (b2 > 0))


def test_linear_regime_is_a_matrix_product():
    # positive weights and inputs keep every unit active: y = x W1 W2 W3 + ...
    rng = np.random.default_rng(3)
    W1 = rng.uniform(0.1, 1.0, (24, 64))
    b1 = rng.uniform(0.1, 1.0, 64)
    W2 = rng.uniform(0.1, 1.0, (64, 64))
    b2 = rng.uniform(0.1, 1.0, 64)
    W3 = rng.normal(size=64)
    b3 = -3.0
    w = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = rng.uniform(0.0, 1.0, (9, 24))
    expect = ((X @ W1 + b1) @ W2 + b2) @ W3 + b3
    assert np.allclose(mlp.forward(w, X), expect)


def test_adam_first_step_is_a_signed_learning_rate():
    rng = np.random.default_rng(4)
    w = rng.normal(size=100)
    g = rng.normal(size=100)
    g[::7] = 0.0
    w1, m1, m2 = mlp.adam_step(w, np.zeros(100), np.zeros(100), g, 1e-3, 1)
    assert np.allclose(w1 - w, -1e-3 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)
    # a constant gradient keeps the bias-corrected step at lr * sign(g)
    w2, m1, m2 = mlp.adam_step(w1, m1, m2, g, 1e-3, 2)
    assert np.allclose(w2 - w1, -1e-3 * g / (np.abs(g) + 1e-8))


def test_bf16_rounding_exact_values_and_ties():
    # values with 8 significant bits are unchanged
    exact = np.array([1.0, -2.5, 0.0078125, 3.0e38, 255.0], dtype=np.float32)
    exact = exact.view(np.uint32) & np.uint32(0xFFFF0000)
    exact = exact.view(np.float32)
    assert np.array_equal(mlp.bf16_round(exact), exact.astype(np.float64))
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even (1.0)
    assert mlp.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6
    # just above a tie rounds up, just below rounds down
    up = np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)
    dn = np.float32(1.0 + 2.0 ** -8 - 2.0 ** -20)
    assert mlp.bf16_round(up) == 1.0 + 2.0 ** -7
    assert mlp.bf16_round(dn) == 1.0
    # 8 significant bits: the rounding error is at most half a unit, 2^-8 relative
    rng = np.random.default_rng(5)
    a = rng.normal(size=10000).astype(np.float32)
    r = mlp.bf16_round(a)
    assert np.all(np.abs(r - a) <= np.abs(a) * 2.0 ** -8)


def test_bf16_inference_rounds_every_product_operand():
    # one active path: x0 -> unit 0 -> unit 0 -> y, every weight 1 (exact in
    # bfloat16) and b3 = 0; the biases are powers of two (also exact). Near 1
    # the bfloat16 values are 2^-7 apart, so the midpoints sit at odd
    # multiples of 2^-8. Values derived by hand:
    def net(b1, b2):
        W1 = np.zeros((mlp.N_IN, mlp.N_HID))
        W2 = np.zeros((mlp.N_HID, mlp.N_HID))
        W3 = np.zeros(mlp.N_HID)
        bb1 = np.zeros(mlp.N_HID)
        bb2 = np.zeros(mlp.N_HID)
        W1[0, 0] = W2[0, 0] = W3[0] = 1.0
        bb1[0], bb2[0] = b1, b2
        return mlp.pack(W1, bb1, W2, bb2, W3, 0.0)

    X = np.zeros((2, mlp.N_IN))
    X[0, 0] = 1.0
    X[1, 0] = 1.0 + 2.0 ** -8 - 2.0 ** -9  # below the midpoint: the input rounds to 1.0
    # h1 = 1 + 2^-9 rounds down to 1; h2 = 1 + 2^-9 rounds down to 1: y = 1
    w = net(2.0 ** -9, 2.0 ** -9)
    assert mlp.forward(w, X[:1])[0] == 1.0 + 2.0 ** -8  # fp64: nothing rounded
    y = mlp.forward_bf16(w, X)
    assert y[0] == 1.0 and y[1] == 1.0
    # h1 = 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: the even one,
    # 1 + 2^-6, goes on; h2 = 1 + 2^-6 + 2^-9 rounds back down to 1 + 2^-6
    assert mlp.forward_bf16(net(3 * 2.0 ** -8, 2.0 ** -9), X[:1])[0] == 1.0 + 2.0 ** -6
    # h1 rounds to 1; h2 = 1 + 2^-8 + 2^-10 is past the midpoint: 1 + 2^-7
    assert mlp.forward_bf16(net(2.0 ** -9, 2.0 ** -8 + 2.0 ** -10), X[:1])[0] == 1.0 + 2.0 ** -7
    # h2 = 1 + 2^-8 exactly (a tie) goes to the even neighbour 1.0
    assert mlp.forward_bf16(net(2.0 ** -9, 2.0 ** -8), X[:1])[0] == 1.0
