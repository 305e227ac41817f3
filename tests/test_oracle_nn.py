"""Pins of the oracle's convolutional network: closed forms of the 3x3
cross-correlation (impulse response, scipy's correlate2d for one channel),
central differences of the loss, and the first Adam step."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn


def test_conv_impulse_response():
    """An impulse at (y0, x0) in channel i reads out the kernel, flipped in
    position: Z[y0-dy+1, x0-dx+1, o] = W[dy, dx, i, o] + b[o]."""
    rng = np.random.default_rng(0)
    W = rng.standard_normal((3, 3, 2, 3))
    b = rng.standard_normal(3)
    A = np.zeros((1, 7, 6, 2))
    A[0, 3, 2, 1] = 1.0
    Z = nn.conv3x3(A, W, b)
    for dy in range(3):
        for dx in range(3):
            assert np.allclose(Z[0, 3 - dy + 1, 2 - dx + 1], W[dy, dx, 1] + b, rtol=0, atol=1e-15)
    # away from the impulse only the bias remains
    assert np.allclose(Z[0, 0, 5], b)


def test_conv_single_channel_is_correlate2d():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((9, 11))
    K = rng.standard_normal((3, 3))
    Z = nn.conv3x3(A[None, :, :, None], K[:, :, None, None], np.zeros(1))[0, :, :, 0]
    ref = correlate2d(A, K, mode="same", boundary="fill", fillvalue=0.0)
    assert np.allclose(Z, ref, rtol=1e-13, atol=1e-13)


def _tiny():
    rng = np.random.default_rng(2)
    sizes = [3, 4, 4, 2]
    params = nn.init_params(sizes, seed=3)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    X = rng.standard_normal((2, 5, 6, 3))
    T = rng.standard_normal((2, 5, 6, 2))
    env = rng.uniform(0.2, 1.0, (5, 6))
    osc = np.array([0.5, 2.0])
    return sizes, params, X, T, env, osc


def test_gradients_match_central_differences():
    sizes, params, X, T, env, osc = _tiny()
    loss, grads = nn.loss_and_grads(params, X, T, env, osc)
    g = nn.flatten(grads)
    p0 = nn.flatten(params)
    rng = np.random.default_rng(4)
    idx = rng.choice(p0.size, 40, replace=False)
    h = 1e-6
    for q in idx:
        pp, pm = p0.copy(), p0.copy()
        pp[q] += h
        pm[q] -= h
        lp, _ = nn.loss_and_grads(nn.unflatten(pp, sizes), X, T, env, osc)
        lm, _ = nn.loss_and_grads(nn.unflatten(pm, sizes), X, T, env, osc)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(abs(fd), 1e-3), (q, fd, g[q])


def test_loss_is_zero_at_an_exact_fit_and_prediction_scales():
    sizes, params, X, T, env, osc = _tiny()
    U = nn.predict(params, X, env, osc)
    loss, grads = nn.loss_and_grads(params, X, U, env, osc)
    assert loss < 1e-28
    assert max(np.abs(nn.flatten(grads)).max(), 0.0) < 1e-13


def test_first_adam_step_moves_by_lr_times_sign():
    """From zero moments the bias-corrected step is lr * g / (|g| + eps)."""
    params = [(np.array([[[[1.0, -2.0]]]]).repeat(3, 0).repeat(3, 1), np.array([0.5, 0.0]))]
    grads = [(np.full((3, 3, 1, 2), 3.0), np.array([-4.0, 1e-3]))]
    state = {}
    new = nn.adam_step(params, grads, state, lr=0.01)
    assert np.allclose(new[0][0], params[0][0] - 0.01 * 3.0 / (3.0 + 1e-8), rtol=1e-15)
    assert new[0][1][0] == pytest.approx(0.5 + 0.01 * 4.0 / (4.0 + 1e-8), rel=1e-15)
    assert new[0][1][1] == pytest.approx(-0.01 * 1e-3 / (1e-3 + 1e-8), rel=1e-12)
    assert state["t"] == 1


def test_flatten_roundtrip():
    sizes, params, *_ = _tiny()
    back = nn.unflatten(nn.flatten(params), sizes)
    for (W, b), (W2, b2) in zip(params, back):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)


def test_input_channels_mean_is_lognormal_mean_by_quadrature():
    """c0 = E[exp(g0 + g . xi)] for standard Gaussian xi: Gauss-Hermite."""
    from numpy.polynomial.hermite_e import hermegauss
    rng = np.random.default_rng(4)
    g0 = 0.2 * rng.standard_normal(5)
    g = 0.4 * rng.standard_normal((2, 5))
    X = nn.input_channels(g0, g)
    x, w = hermegauss(30)
    w = w / w.sum()
    for p in range(5):
        q = sum(wa * wb * np.exp(g0[p] + g[0, p] * xa + g[1, p] * xb)
                for xa, wa in zip(x, w) for xb, wb in zip(x, w))
        assert X[p, 0] == pytest.approx(q, rel=1e-13)
    assert np.array_equal(X[:, 1:], g.T)


def test_output_map_closed_forms():
    """Constant targets c_k give oscale_k = |c_k| / RMS(env); env peaks at 1."""
    shape = np.array([1.0, 3.0, 2.0, 4.0])
    T = np.empty((3, 4, 2))
    T[..., 0] = -2.0
    T[..., 1] = 0.5
    env, osc = nn.output_map(shape, T)
    assert np.allclose(env, [0.25, 0.75, 0.5, 1.0]) and env.max() == 1.0
    rms_env = np.sqrt((0.25 ** 2 + 0.75 ** 2 + 0.5 ** 2 + 1.0) / 4)
    assert np.allclose(osc, [2.0 / rms_env, 0.5 / rms_env], rtol=1e-15)
