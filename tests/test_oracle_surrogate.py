"""Pins of the surrogate network's FP64 reference (oracle/surrogate.py)."""
import numpy as np
import pytest
from scipy.signal import correlate2d


def test_depthwise_conv_matches_library_correlation():
    from oracle import surrogate as S

    rng = np.random.default_rng(0)
    h = rng.standard_normal((2, 9, 11, 4))
    k = rng.standard_normal((4, 3, 3))
    b = rng.standard_normal(4)
    out = S.dw3x3(h, k, b)
    for n in range(2):
        for c in range(4):
            ref = correlate2d(h[n, :, :, c], k[c], mode="same", boundary="fill") + b[c]
            assert np.allclose(out[n, :, :, c], ref, rtol=1e-13, atol=1e-13)


def test_depthwise_conv_backward_is_transpose():
    from oracle import surrogate as S

    rng = np.random.default_rng(1)
    h = rng.standard_normal((1, 7, 8, 3))
    k = rng.standard_normal((3, 3, 3))
    d = rng.standard_normal(h.shape)
    dh, dk, db = S.dw3x3_backward(h, k, d)
    # <dw(h), d> is linear in h and in k: compare with the adjoint identities
    lhs = np.sum((S.dw3x3(h, k, np.zeros(3))) * d)
    assert lhs == pytest.approx(np.sum(h * dh), rel=1e-12)
    assert lhs == pytest.approx(np.sum(k * dk), rel=1e-12)
    assert np.allclose(db, d.sum(axis=(0, 1, 2)))


def test_gelu_derivative():
    from oracle import surrogate as S

    p = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (S.gelu(p + h) - S.gelu(p - h)) / (2 * h)
    assert np.allclose(S.gelu_grad(p), fd, rtol=1e-8, atol=1e-9)
    assert S.gelu(np.array([0.0]))[0] == 0.0


def test_bf16_rounding():
    from oracle import surrogate as S

    assert S.bf(1.0 + 2.0 ** -9) == 1.0            # below half an ulp (2^-8)
    assert S.bf(1.0 + 3 * 2.0 ** -9) == 1.0 + 2.0 ** -7
    assert S.bf(1.0 + 2.0 ** -8) == 1.0            # tie to even
    assert S.bf(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie to even (odd mantissa rounds up)


@pytest.fixture(scope="module")
def small_problem():
    from oracle import surrogate as S
    import fwi_inputs as fi

    params = S.init_params(3)
    v = fi.faulted_model(70, 70, 5)[None]
    rng = np.random.default_rng(4)
    Rw = rng.standard_normal((1, S.NS, S.NR, S.NT))
    return S, params, v, Rw


def test_backward_input_gradient_fd(small_problem):
    """d/dv of <traces(v), R> by the chain rule equals central differences (FP64)."""
    S, params, v, Rw = small_problem
    tr, cache = S.forward(params, v, rounding=False)
    dv, _ = S.backward(params, cache, Rw)
    rng = np.random.default_rng(5)
    for _ in range(2):
        dirn = rng.standard_normal(v.shape)
        h = 1e-3
        fp = np.sum(S.forward(params, v + h * dirn, rounding=False)[0] * Rw)
        fm = np.sum(S.forward(params, v - h * dirn, rounding=False)[0] * Rw)
        fd = (fp - fm) / (2 * h)
        assert np.sum(dv * dirn) == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("name,idx", [("enc1_w1", (3, 7)), ("dec2_xm", (10, 40)), ("dec3_dw_k", (5, 1, 2)),
                                      ("d2t", (100, 20)), ("up", (500, 60)), ("lift_w", (0, 9)),
                                      ("enc0_b2", (4,)), ("proj_w", (12, 3))])
def test_backward_weight_gradients_fd(small_problem, name, idx):
    S, params, v, Rw = small_problem
    tr, cache = S.forward(params, v, rounding=False)
    _, grads = S.backward(params, cache, Rw)
    h = 1e-5 * max(1.0, abs(params[name][idx]))
    pp = {k: (a.copy() if isinstance(a, np.ndarray) else a) for k, a in params.items()}
    pm = {k: (a.copy() if isinstance(a, np.ndarray) else a) for k, a in params.items()}
    pp[name][idx] += h
    pm[name][idx] -= h
    fd = (np.sum(S.forward(pp, v, rounding=False)[0] * Rw) - np.sum(S.forward(pm, v, rounding=False)[0] * Rw)) / (2 * h)
    assert grads[name][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9 * max(1.0, abs(fd)))
