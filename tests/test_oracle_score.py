"""Pins of the score network's FP64 reference (oracle/score.py): the 3 x 3
convolution against a library correlation, every transpose against its
forward by the adjoint identity, the whole backward pass and the denoising
score-matching gradient against central finite differences, and the output
map (noise, score, clean estimate of Eq. v0hat)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import score as S


def test_conv3_im2col_matches_library_correlation():
    rng = np.random.default_rng(0)
    h = rng.standard_normal((2, 9, 9, 3))
    Wt = rng.standard_normal((9 * 3, 4))
    out = S.im2col(h) @ Wt
    for n in range(2):
        for co in range(4):
            ref = np.zeros((9, 9))
            for ci in range(3):
                k = np.array([[Wt[(3 * dy + dx) * 3 + ci, co] for dx in range(3)] for dy in range(3)])
                ref += correlate2d(h[n, :, :, ci], k, mode="same", boundary="fill")
            assert np.allclose(out[n, :, :, co], ref, rtol=1e-12, atol=1e-12)


def test_transposes():
    rng = np.random.default_rng(1)
    h = rng.standard_normal((2, 8, 8, 3))
    d = rng.standard_normal((2, 8, 8, 27))
    assert np.sum(S.im2col(h) * d) == pytest.approx(np.sum(h * S.col2im(d, 3)), rel=1e-12)
    y = rng.standard_normal((2, 4, 4, 3))
    assert np.sum(S.up2(y) * h) == pytest.approx(np.sum(y * S.up2_transpose(h)), rel=1e-12)
    assert np.sum(S.pool(h) * y) == pytest.approx(np.sum(h * 0.25 * S.up2(y)), rel=1e-12)
    assert np.allclose(S.pool(S.up2(y)), y)


def test_time_features():
    e = S.time_features([0.0, 0.5])
    assert np.all(e[0, :S.NF] == 0.0) and np.all(e[0, S.NF:] == 1.0)
    assert e[1, 0] == pytest.approx(np.sin(500.0)) and e[1, S.NF] == pytest.approx(np.cos(500.0))
    assert S.param_count() == sum(np.prod(s) for _, s in S.layout())


@pytest.fixture(scope="module")
def net():
    p = S.init_params(7)
    rng = np.random.default_rng(3)
    for n in p:   # non-zero biases so that every term is exercised
        if p[n].ndim == 1:
            p[n] = 0.1 * rng.standard_normal(p[n].shape)
    x = rng.uniform(-1, 1, (2, 70, 70))
    t = np.array([0.31, 0.77])
    return p, x, t


def test_output_map(net):
    p, x, t = net
    eps, _ = S.forward(p, x, t, rounding=False)
    out, _ = S.forward(p, x, t, skip=[0.5, -2.0], scale=[3.0, 0.25], rounding=False)
    assert np.allclose(out[0], 0.5 * x[0] + 3.0 * eps[0], rtol=1e-13, atol=1e-13)
    assert np.allclose(out[1], -2.0 * x[1] + 0.25 * eps[1], rtol=1e-13, atol=1e-13)


def test_input_vjp_matches_finite_differences(net):
    p, x, t = net
    rng = np.random.default_rng(4)
    skip, scale = np.array([0.3, 1.1]), np.array([-1.7, 0.6])
    a = rng.standard_normal(x.shape)
    dirn = rng.standard_normal(x.shape)
    _, cache = S.forward(p, x, t, skip=skip, scale=scale, rounding=False)
    dx, _ = S.backward(p, cache, a)
    h = 1e-5
    fp = np.sum(S.forward(p, x + h * dirn, t, skip=skip, scale=scale, rounding=False)[0] * a)
    fm = np.sum(S.forward(p, x - h * dirn, t, skip=skip, scale=scale, rounding=False)[0] * a)
    fd = (fp - fm) / (2 * h)
    assert np.sum(dx * dirn) == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("group", ["temb", "lift", "b0a", "down0", "b1a", "down1", "b2", "up1", "b1b", "up0",
                                   "b0b", "head"])
def test_parameter_gradients_match_finite_differences(net, group):
    p, x, t = net
    rng = np.random.default_rng(hash(group) % 1000)
    a = rng.standard_normal(x.shape)
    _, cache = S.forward(p, x, t, rounding=False)
    _, g = S.backward(p, cache, a)
    names = [n for n, _ in S.layout() if n.startswith(group + "_")]
    assert names
    dirn = {n: rng.standard_normal(p[n].shape) for n in names}
    h = 1e-6

    def f(sign):
        q = dict(p)
        for n in names:
            q[n] = p[n] + sign * h * dirn[n]
        return np.sum(S.forward(q, x, t, rounding=False)[0] * a)

    fd = (f(1) - f(-1)) / (2 * h)
    an = sum(np.sum(g[n] * dirn[n]) for n in names)
    assert an == pytest.approx(fd, rel=2e-6, abs=1e-9 * abs(fd) + 1e-12)


def test_dsm_loss_gradient(net):
    p, _, _ = net
    rng = np.random.default_rng(9)
    beta = np.linspace(1e-4, 0.02, 1000)
    abar = np.cumprod(1 - beta)
    x0 = rng.uniform(-1, 1, (2, 70, 70))
    noise = rng.standard_normal((2, 70, 70))
    ti = np.array([120, 870])
    loss, g = S.dsm_loss(p, x0, noise, ti, abar, rounding=False)
    dirn = {n: rng.standard_normal(p[n].shape) for n in p}
    h = 1e-6
    lp = S.dsm_loss({n: p[n] + h * dirn[n] for n in p}, x0, noise, ti, abar, rounding=False)[0]
    lm = S.dsm_loss({n: p[n] - h * dirn[n] for n in p}, x0, noise, ti, abar, rounding=False)[0]
    assert sum(np.sum(g[n] * dirn[n]) for n in p) == pytest.approx((lp - lm) / (2 * h), rel=1e-6)
    # the loss is the mean squared noise-prediction error at the noised states
    ab = abar[ti - 1]
    xt = np.sqrt(ab)[:, None, None] * x0 + np.sqrt(1 - ab)[:, None, None] * noise
    eps, _ = S.forward(p, xt, ti / 1000.0, rounding=False)
    assert loss == pytest.approx(np.mean((eps - noise) ** 2), rel=1e-12)
