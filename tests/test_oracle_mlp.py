"""Pins of the CPU multilayer-perceptron reference (oracle/mlp.py)."""
import numpy as np

from oracle import mlp as M


def _net(seed=0, widths=(3, 7, 5, 4)):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(M.param_count(widths)) * 0.4
    x = rng.standard_normal((6, widths[0]))
    t = rng.standard_normal((6, widths[-1]))
    return widths, p, x, t


def test_gradient_matches_central_differences():
    widths, p, x, t = _net()
    loss, g = M.loss_and_grad(p, widths, x, t, bf16=False)
    h = 1e-6
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = M.loss_and_grad(p + e, widths, x, t, bf16=False)
        lm, _ = M.loss_and_grad(p - e, widths, x, t, bf16=False)
        assert abs((lp - lm) / (2 * h) - g[i]) < 1e-7 * max(1.0, abs(g[i]))


def test_packing_layout():
    widths = (2, 3, 1)
    assert M.param_count(widths) == 2 * 3 + 3 + 3 * 1 + 1
    p = np.arange(M.param_count(widths), dtype=float)
    (W0, b0), (W1, b1) = M.unpack(p, widths)
    assert W0.shape == (3, 2) and W0[1, 0] == 2 and b0[0] == 6 and W1[0, 2] == 11 and b1[0] == 12


def test_bf16_rounding():
    exact = np.array([1.0, -2.5, 0.15625, 65280.0], dtype=np.float32)   # representable in bf16
    assert np.array_equal(M.bf16_round(exact), exact.astype(np.float64))
    one = np.float32(1.0)
    ulp = 2.0 ** -7                                     # bf16 spacing at 1
    half = np.float32(1.0 + ulp / 2)                    # tie: rounds to even (1.0)
    above = np.float32(1.0 + ulp / 2 + 2.0 ** -20)      # just above the tie
    three_half = np.float32(1.0 + 3 * ulp / 2)          # tie between 1+ulp (odd) and 1+2ulp (even)
    assert M.bf16_round(half) == one
    assert M.bf16_round(above) == 1.0 + ulp
    assert M.bf16_round(three_half) == 1.0 + 2 * ulp
    rng = np.random.default_rng(3)
    v = rng.standard_normal(1000).astype(np.float32)
    r = M.bf16_round(v)
    assert np.all(np.abs(r - v) <= np.abs(v) * 2.0 ** -8 * 1.0000001)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p, g = rng.standard_normal(10), rng.standard_normal(10)
    z = np.zeros(10)
    q, m, v = M.adam(p, z, z, g, 1, lr=0.01, eps=0.0)
    # after one step the bias-corrected moments are g and g^2, so the step is lr * sign(g)
    assert np.allclose(q, p - 0.01 * np.sign(g))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
