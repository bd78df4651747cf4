"""Pins of the surrogate's FP64 oracle: convolution against scipy's correlate2d,
gradients against central finite differences, BF16 rounding against its bit
definition, Adam against a hand-computed first step."""
import numpy as np
import pytest

from oracle import surrogate_oracle as S


def test_conv3x3_matches_scipy_correlate():
    from scipy.signal import correlate2d
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 7, 9))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    y = S.conv3x3(x, W, b)
    for o in range(2):
        ref = b[o] + sum(correlate2d(x[c], W[o, c], mode="same", boundary="fill")
                         for c in range(3))
        np.testing.assert_allclose(y[o], ref, rtol=1e-13, atol=1e-13)


def test_conv3x3_single_tap_is_a_shift():
    x = np.arange(20.0).reshape(1, 4, 5)
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 0, 2] = 1.0          # weight at (di, dj) = (0, 2): reads x[i-1, j+1]
    y = S.conv3x3(x, W, np.zeros(1))
    assert y[0, 1, 0] == x[0, 0, 1] and y[0, 0, 0] == 0.0 and y[0, 3, 4] == 0.0


def _loss(x, Ws, bs, target):
    out, _ = S.forward(x, Ws, bs, bf16=False)
    return S.mse(out, target)[0]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    chans = (2, 4, 3, 2)
    Ws, bs = S.init_weights(chans, seed=3)
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    x = rng.standard_normal((2, 5, 6))
    target = rng.standard_normal((2, 5, 6))
    out, cache = S.forward(x, Ws, bs, bf16=False)
    _, dout = S.mse(out, target)
    gW, gb = S.backward(Ws, cache, dout, bf16=False)
    h = 1e-6
    for l in range(len(Ws)):
        for idx in [(0, 0, 1, 1), (1, 0, 2, 0), (0, 1, 0, 2)]:
            if idx[0] >= Ws[l].shape[0] or idx[1] >= Ws[l].shape[1]:
                continue
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (_loss(x, Wp, bs, target) - _loss(x, Wm, bs, target)) / (2 * h)
            assert gW[l][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][0] += h
        bm[l][0] -= h
        fd = (_loss(x, Ws, bp, target) - _loss(x, Ws, bm, target)) / (2 * h)
        assert gb[l][0] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_input_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 4, 4))
    W = rng.standard_normal((2, 3, 3, 3))
    dy = rng.standard_normal((2, 4, 4))
    dx, _, _ = S.conv3x3_backward(x, W, dy)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (2, 3, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (np.sum(dy * S.conv3x3(xp, W, np.zeros(2))) -
              np.sum(dy * S.conv3x3(xm, W, np.zeros(2)))) / (2 * h)
        assert dx[idx] == pytest.approx(fd, rel=1e-6)


def test_bf16_rounding_bits():
    # 1 + 2^-8 is exactly halfway between two bf16 values: ties to even -> 1.0
    assert S.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    # 1 + 3*2^-8 is halfway between 1+2^-7 and 1+2^-6: ties to even -> 1 + 2^-6
    assert S.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6
    assert S.bf16_round(np.float32(1.0 + 2 ** -7)) == 1.0 + 2 ** -7
    assert S.bf16_round(np.float32(-3.0)) == -3.0
    x = np.random.default_rng(0).standard_normal(1000)
    r = S.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8)


def test_adam_first_step():
    """Adam's bias-corrected first step moves each parameter by lr * sign(g)
    (up to eps): m_hat = g, v_hat = g^2."""
    p = [np.array([1.0, -2.0])]
    g = [np.array([0.5, -4.0])]
    m = [np.zeros(2)]
    v = [np.zeros(2)]
    S.adam_step(p, g, m, v, t=1, lr=0.01)
    np.testing.assert_allclose(p[0], [1.0 - 0.01, -2.0 + 0.01], rtol=0, atol=1e-8)
    np.testing.assert_allclose(m[0], [0.05, -0.4])
    np.testing.assert_allclose(v[0], [0.00025, 0.016])
