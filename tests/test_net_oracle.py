"""Pins of the network oracle: library correlation, identity kernel,
adjointness of pooling/upsampling, finite-difference gradients, and the
bfloat16 rounding rule.  CPU only."""
import numpy as np
import pytest
from scipy import signal

from oracle import net_oracle as N


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 6, 7))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    y = N.conv(x, w, b)
    for o in range(2):
        ref = b[o] + sum(signal.correlate(x[c], w[o, c], mode="same") for c in range(3))
        assert np.allclose(y[o], ref, rtol=0, atol=1e-12)


def test_delta_kernel_is_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 4, 4, 4))
    w = np.zeros((4, 4, 3, 3, 3))
    for c in range(4):
        w[c, c, 1, 1, 1] = 1.0
    assert np.array_equal(N.conv(x, w, np.zeros(4)), x)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 6, 8))
    y = rng.standard_normal((3, 2, 3, 4))
    # <pool x, y> = <x, pool^T y>; <up y, x> = <y, up^T x>
    assert abs(np.sum(N.pool(x) * y) - np.sum(x * N.pool_backward(y))) < 1e-12
    assert abs(np.sum(N.up(y) * x) - np.sum(y * N.up_backward(x))) < 1e-12
    assert np.allclose(N.pool(N.up(y)), y)


def test_conv_backward_adjoint():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 4, 5, 6))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    dy = rng.standard_normal((2, 4, 5, 6))
    dx, dw, db = N.conv_backward(x, w, dy)
    # linear in x: <conv(x) - b, dy> = <x, dx>
    assert abs(np.sum((N.conv(x, w, np.zeros(2))) * dy) - np.sum(x * dx)) < 1e-10
    # linear in w: <conv_w(x), dy> = <w, dw>
    assert abs(np.sum(N.conv(x, w, np.zeros(2)) * dy) - np.sum(w * dw)) < 1e-10
    assert np.allclose(db, dy.sum(axis=(1, 2, 3)))


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    theta = N.he_init(5) * 0.7
    theta[-161:] = rng.standard_normal(161) * 0.1         # nonzero biases
    feat = rng.standard_normal((4, 4, 4, 8))
    target = rng.standard_normal((4, 4, 8)) * 0.1
    P = N.unflatten(theta)
    out, cache = N.forward(P, feat)
    L, dout = N.loss_and_grad(out, target)
    g = N.flatten(N.backward(cache, dout))
    idx = rng.choice(theta.size, 60, replace=False)
    idx = np.concatenate([idx, np.arange(theta.size - 161, theta.size, 17)])
    eps = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += eps
        tm[i] -= eps
        Lp = N.loss_and_grad(N.forward(N.unflatten(tp), feat)[0], target)[0]
        Lm = N.loss_and_grad(N.forward(N.unflatten(tm), feat)[0], target)[0]
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_bf16_rounding_rule():
    # exactly representable values are unchanged
    v = np.array([1.0, -2.5, 0.0, 65280.0, 2.0 ** -10])
    assert np.array_equal(N.bf16_round(v), v)
    # halfway cases go to the even mantissa
    one = np.float32(1.0)
    half_ulp = np.float32(2.0 ** -8)      # bf16 has 8 significand bits incl. the implicit one
    assert N.bf16_round(one + half_ulp) == 1.0
    assert N.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 4 * 2.0 ** -8
    # relative error bound 2^-9
    x = np.random.default_rng(6).standard_normal(10000)
    assert np.max(np.abs(N.bf16_round(x) - x) / np.abs(x)) <= 2.0 ** -8


def test_adam_first_step_moves_by_lr():
    th = np.zeros(5)
    g = np.array([1.0, -2.0, 3.0, -4.0, 0.5])
    th1, m, v = N.adam_step(th, g, np.zeros(5), np.zeros(5), 1, lr=1e-3)
    assert np.allclose(th1, -1e-3 * np.sign(g), rtol=1e-6)


def test_param_count():
    assert N.param_count() == (16 * 4 * 27 + 16) + (32 * 16 * 27 + 32) + (64 * 32 * 27 + 64) + \
        (32 * 96 * 27 + 32) + (16 * 48 * 27 + 16) + (16 + 1)


def test_energy_loss_gradient_and_special_values():
    rng = np.random.default_rng(8)
    n = 30
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)                     # SPD
    op = lambda x: (A @ x.ravel()).reshape(x.shape)
    t = rng.standard_normal((2, 3, 5))
    d = rng.standard_normal((2, 3, 5))
    L, g = N.energy_loss_and_grad(d, t, op)
    assert abs(N.energy_loss_and_grad(np.zeros_like(t), t, op)[0] - 1.0) < 1e-14   # delta = 0 is p_prev
    assert N.energy_loss_and_grad(t, t, op)[0] == 0.0                             # exact guess
    eps = 1e-6
    for idx in [(0, 0, 0), (1, 2, 4), (0, 1, 3)]:
        dp = d.copy()
        dm = d.copy()
        dp[idx] += eps
        dm[idx] -= eps
        fd = (N.energy_loss_and_grad(dp, t, op)[0] - N.energy_loss_and_grad(dm, t, op)[0]) / (2 * eps)
        assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(fd))


def test_bf16_emulation_stays_within_rounding_of_the_exact_network():
    """The bfloat16 emulation rounds (features, 3x3x3 weights, activations and
    activation gradients) but keeps the head in full precision: with inputs
    and weights that are already bfloat16 numbers, its output and gradients
    stay within a few bfloat16 roundings (2^-8 relative each, compounded over
    the layers) of the FP64 network's, and differ from them (something is
    rounded).  A head whose weights are bfloat16 numbers and a loss gradient
    that is one make the two heads' arithmetic identical, so any difference
    comes from the emulated storage."""
    rng = np.random.default_rng(31)
    theta = N.bf16_round(N.he_init(5))
    theta[-17:] = N.bf16_round(rng.standard_normal(17) * 0.3)
    P = N.unflatten(theta)
    feat = N.bf16_round(rng.standard_normal((4, 8, 8, 8)))
    out64, c64 = N.forward(P, feat)
    out16, c16 = N.forward(P, feat, bf16=True)
    r_out = np.linalg.norm(out16 - out64) / np.linalg.norm(out64)
    assert 1e-5 < r_out < 3e-2
    dout = N.bf16_round(rng.standard_normal(out64.shape))
    g64 = N.backward(c64, dout)
    g16 = N.backward(c16, dout)
    for k in g64:
        r = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
        assert r < 6e-2, k
    # the head's weight gradient sees only a5, rounded the same way on both
    # paths up to the activations' own rounding; the deepest gradient (c1)
    # has passed through every rounded tensor
    r_c1 = np.linalg.norm(g16["c1.w"] - g64["c1.w"]) / np.linalg.norm(g64["c1.w"])
    assert r_c1 > 1e-4
