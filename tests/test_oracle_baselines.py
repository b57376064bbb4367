"""Pins of the oracle's least-squares potential (Phi_l2 of baseline DPS, Sec. 4
and the MSE ablation of Sec. 6) and of its total-variation subgradient
(Eq. tv, used by the TV-regularised baselines of Sec. 6).

Each check is independent of the oracle's own formula: finite differences of
J for the adjoint source, closed forms for a constant shift and for a single
spike at the observation maximum (which fixes the weight 1/(1 + k)),
invariance of the normalised potential under a common rescaling, the
subgradient inequality of the convex TV against a separate numpy TV, and
exact directional derivatives of the piecewise-linear TV at a generic point.
"""
import numpy as np
import pytest

import oracle


def _traces(seed, shape=(2, 3, 40)):
    rng = np.random.default_rng(seed)
    t = np.arange(shape[-1])
    env = np.exp(-0.5 * ((t - 15) / 6.0) ** 2)
    return rng.standard_normal(shape) * env


def test_l2_constant_shift_closed_form():
    d_obs = _traces(0)
    c, sigma = 0.3, 0.05
    J, adj = oracle.l2_misfit(d_obs + c, d_obs, sigma=sigma)
    n = d_obs.size
    assert J == pytest.approx(0.5 * c * c * n / sigma ** 2, rel=1e-12)
    assert np.allclose(adj, c / sigma ** 2, rtol=1e-12)


def test_l2_single_spike_weight():
    """One observed spike of amplitude A (the maximum, so a = 1 there): a
    residual r at that sample costs (r / (1 + k))^2 / (2 sigma^2); at a zero
    observation the weight is 1."""
    d_obs = np.zeros((1, 2, 10))
    d_obs[0, 1, 4] = -2.5
    k, sigma, r = 100.0, 0.5, 0.7
    d = d_obs.copy()
    d[0, 1, 4] += r
    J, adj = oracle.l2_misfit(d, d_obs, sigma=sigma, k=k)
    assert J == pytest.approx(0.5 * (r / (1 + k)) ** 2 / sigma ** 2, rel=1e-12)
    assert adj[0, 1, 4] == pytest.approx(r / (1 + k) ** 2 / sigma ** 2, rel=1e-12)
    d2 = d_obs.copy()
    d2[0, 0, 3] = r
    J2, _ = oracle.l2_misfit(d2, d_obs, sigma=sigma, k=k)
    assert J2 == pytest.approx(0.5 * r * r / sigma ** 2, rel=1e-12)


@pytest.mark.parametrize("k,normalize", [(0.0, False), (100.0, False), (0.0, True), (100.0, True), (3.0, True)])
def test_l2_adjoint_is_the_derivative(k, normalize):
    d_obs = _traces(1)
    d_syn = np.stack([d_obs + 0.2 * _traces(s) for s in (2, 3)])
    J, adj = oracle.l2_misfit(d_syn, d_obs, sigma=0.05, k=k, normalize=normalize)
    rng = np.random.default_rng(4)
    h = 1e-6
    for _ in range(12):
        b = rng.integers(2)
        idx = tuple(rng.integers(s) for s in d_obs.shape)
        dp, dm = d_syn.copy(), d_syn.copy()
        dp[(b,) + idx] += h
        dm[(b,) + idx] -= h
        Jp, _ = oracle.l2_misfit(dp, d_obs, sigma=0.05, k=k, normalize=normalize, want_adjoint=False)
        Jm, _ = oracle.l2_misfit(dm, d_obs, sigma=0.05, k=k, normalize=normalize, want_adjoint=False)
        fd = (Jp[b] - Jm[b]) / (2 * h)
        assert fd == pytest.approx(adj[(b,) + idx], rel=1e-6, abs=1e-9 * max(1.0, abs(J[b])))
    # the other sample's J does not move
    assert J.shape == (2,)


def test_l2_normalised_is_scale_invariant_and_zero_at_the_data():
    d_obs = _traces(5)
    d_syn = d_obs + 0.1 * _traces(6)
    for k in (0.0, 50.0):
        J1, _ = oracle.l2_misfit(d_syn, d_obs, k=k, normalize=True)
        J2, _ = oracle.l2_misfit(7.5 * d_syn, 7.5 * d_obs, k=k, normalize=True)
        assert J1 == pytest.approx(J2, rel=1e-12)
        J0, adj0 = oracle.l2_misfit(d_obs, d_obs, k=k, normalize=True)
        assert J0 == 0.0 and not np.any(adj0)
    # unweighted and normalised: |r|^2 / (2 |d_obs|^2)
    J, _ = oracle.l2_misfit(d_syn, d_obs, normalize=True)
    assert J == pytest.approx(0.5 * np.sum((d_syn - d_obs) ** 2) / np.sum(d_obs ** 2), rel=1e-12)


def test_l2_zero_observations():
    """All-zero observations: the weight is 1 and the normalising scale falls back to 1."""
    d_obs = np.zeros((2, 5))
    d = np.full((2, 5), 0.5)
    J, adj = oracle.l2_misfit(d, d_obs, k=100.0, normalize=True)
    assert J == pytest.approx(0.5 * 10 * 0.25) and np.allclose(adj, 0.5)


def test_l2_rejects_bad_arguments():
    d = np.zeros((2, 5))
    with pytest.raises(oracle.OracleError):
        oracle.l2_misfit(d, d, sigma=0.0)
    with pytest.raises(oracle.OracleError):
        oracle.l2_misfit(d, d, k=-1.0)


def _tv(x):
    """TV of Eq. tv: mean over the grid of |forward x-difference| + |forward z-difference|."""
    return (np.abs(np.diff(x, axis=1)).sum() + np.abs(np.diff(x, axis=0)).sum()) / x.size


def _fields():
    rng = np.random.default_rng(11)
    yield rng.standard_normal((7, 9))                          # generic: no ties
    x = np.zeros((12, 10))                                     # layers and a step: many ties
    x[4:, :] = 1.0
    x[8:, 5:] = 3.0
    yield x
    yield np.round(rng.standard_normal((6, 6)))                # integer field: ties among neighbours
    yield rng.standard_normal((1, 8))                          # one row: x-differences only
    yield rng.standard_normal((5, 1))                          # one column
    yield np.zeros((3, 3))                                     # flat: subgradient 0


@pytest.mark.parametrize("x", list(_fields()))
def test_tv_subgradient_inequality(x):
    q = oracle.tv_subgradient(x)
    rng = np.random.default_rng(3)
    for _ in range(50):
        y = x + rng.standard_normal(x.shape) * rng.choice([1e-3, 0.1, 2.0])
        assert _tv(y) >= _tv(x) + np.sum(q * (y - x)) - 1e-12


def test_tv_directional_derivative_at_a_generic_point():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, 9, 11))
    q = oracle.tv_subgradient(x)
    for b in range(2):
        for _ in range(10):
            d = rng.standard_normal((9, 11))
            eps = 1e-7
            fd = (_tv(x[b] + eps * d) - _tv(x[b] - eps * d)) / (2 * eps)
            assert fd == pytest.approx(np.sum(q[b] * d), rel=1e-6, abs=1e-12)


def test_tv_subgradient_adds_to_g_and_small_case():
    x = np.array([[0.0, 1.0], [0.0, 0.0]])
    g = np.array([[10.0, 20.0], [30.0, 40.0]])
    out = oracle.tv_subgradient(x, g, alpha=2.0)
    # differences: (0,0)->(0,1): +1; (1,0)->(1,1): 0; (0,0)->(1,0): 0; (0,1)->(1,1): -1; n = 4
    q = np.array([[-1.0, 1.0 + 1.0], [0.0, -1.0]]) / 4.0
    assert np.allclose(out, g + 2.0 * q, rtol=0, atol=1e-15)
