"""Pins of the dense-layer oracle (the warm-start network's layers).

References independent of the oracle's own formulas: forward values by
explicit loops on a tiny case; backward by central finite differences of the
scalar loss sum(G * Y); ADAM's first step in closed form (with eps = 0 each
parameter moves by exactly lr against the sign of its gradient, whatever the
betas); BF16 rounding on hand-worked bit patterns, including both kinds of
ties.
"""
import numpy as np
import pytest

from oracle import mlp


def test_forward_matches_explicit_loops():
    rng = np.random.default_rng(0)
    X, W, b = rng.standard_normal((3, 4)), rng.standard_normal((4, 5)), rng.standard_normal(5)
    for act in (0, 1):
        Y = mlp.forward(X, W, b, act)
        for i in range(3):
            for j in range(5):
                z = b[j]
                for k in range(4):
                    z += X[i, k] * W[k, j]
                assert abs(Y[i, j] - (max(z, 0.0) if act else z)) <= 1e-14


@pytest.mark.parametrize("act", [0, 1])
def test_backward_matches_finite_differences(act):
    rng = np.random.default_rng(1 + act)
    m, k, n = 4, 6, 5
    X, W, b = rng.standard_normal((m, k)), rng.standard_normal((k, n)), rng.standard_normal(n)
    G = rng.standard_normal((m, n))
    Z = X @ W + b
    if act == 1:  # keep every pre-activation away from the ReLU kink
        b = b + np.where(np.abs(Z) < 0.05, 0.2, 0.0).max(axis=0)
    loss = lambda X_, W_, b_: float(np.sum(G * mlp.forward(X_, W_, b_, act)))
    Y = mlp.forward(X, W, b, act)
    dX, dW, db = mlp.backward(X, W, Y, G, act)
    h = 1e-6
    for arr, grad, name in ((X, dX, "X"), (W, dW, "W"), (b, db, "b")):
        num = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            e = np.zeros_like(arr)
            e[idx] = h
            args = {"X": X, "W": W, "b": b}
            args[name] = arr + e
            up = loss(args["X"], args["W"], args["b"])
            args[name] = arr - e
            dn = loss(args["X"], args["W"], args["b"])
            num[idx] = (up - dn) / (2 * h)
        np.testing.assert_allclose(grad, num, atol=1e-7, err_msg=name)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(3)
    p, g = rng.standard_normal(10), rng.standard_normal(10)
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9), (0.0, 0.0)):
        p1, m, v = mlp.adam_step(p, g, np.zeros(10), np.zeros(10), 1, 0.01, b1, b2, 0.0)
        np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    pt, m, v = p.copy(), np.zeros(10), np.zeros(10)
    for t in range(1, 6):
        pt, m, v = mlp.adam_step(pt, g, m, v, t, 0.01, 0.9, 0.999, 0.0)
    np.testing.assert_allclose(pt, p - 5 * 0.01 * np.sign(g), atol=1e-13)


def test_bf16_rounding_bit_patterns():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)  # BF16 spacing at 1
    cases = [
        (one, 0x3F80),
        (one + ulp / 2, 0x3F80),          # tie, 1.0 has an even mantissa: down
        (one + 3 * ulp / 2, 0x3F82),      # tie, 1 + ulp is odd: up to 1 + 2 ulp
        (one + ulp / 2 + np.float32(2.0 ** -20), 0x3F81),  # just above the tie: up
        (np.float32(-2.0), 0xC000),
        (np.float32(0.0), 0x0000),
        (np.float32(3.140625), 0x4049),   # exactly representable
    ]
    for x, bits in cases:
        assert int(mlp.bf16_bits(np.array([x], np.float32))[0]) == bits, (x, hex(bits))
