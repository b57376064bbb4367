"""Pins of the oracle's reverse DDPM step (Algorithm 2: the clean estimator
Eq. v0hat and the posterior-mean-plus-noise line; VP schedule of Sec. 5.3 in
DDPM indexing): closed forms of the forward noising process q(v_i | x0) =
N(sqrt(abar_i) x0, (1 - abar_i) I) that any correct implementation meets.

* with the exact score of q(v_i | x0), -(v_i - sqrt(abar_i) x0)/(1 - abar_i),
  the clean estimator returns x0;
* the posterior-mean coefficients reproduce sqrt(abar_{i-1}) x0 from a
  noise-free state (the mean of q(v_{i-1} | x0));
* they equal the noise-prediction form (v_i - beta_i / sqrt(1 - abar_i) eps) /
  sqrt(alpha_i) of the same mean when v0hat is the estimate implied by eps;
* at i = 1 (abar_0 = 1) the step returns v0hat, and the noise enters as sigma z.
"""
import numpy as np
import pytest

import oracle


def _schedule(N=1000, b0=1e-4, b1=0.02):
    beta = np.linspace(b0, b1, N)
    abar = np.cumprod(1.0 - beta)
    return beta, abar


@pytest.mark.parametrize("i", [1, 2, 10, 500, 999])
def test_exact_score_recovers_x0_and_mean(i):
    beta, abar = _schedule()
    rng = np.random.default_rng(i)
    x0 = rng.standard_normal((3, 7, 5))
    eps = rng.standard_normal(x0.shape)
    ab, abp = abar[i - 1], (abar[i - 2] if i > 1 else 1.0)
    v = np.sqrt(ab) * x0 + np.sqrt(1 - ab) * eps
    s = -(v - np.sqrt(ab) * x0) / (1 - ab)
    v0, vp = oracle.ddpm_step(v, beta[i - 1], ab, abp, score=s)
    assert np.allclose(v0, x0, rtol=0, atol=1e-9 / np.sqrt(ab))
    # noise-prediction form of the posterior mean
    mu = (v - beta[i - 1] / np.sqrt(1 - ab) * eps) / np.sqrt(1 - beta[i - 1])
    assert np.allclose(vp, mu, rtol=0, atol=1e-9 / np.sqrt(ab))
    # a noise-free state maps to the mean of q(v_{i-1} | x0)
    _, vp0 = oracle.ddpm_step(np.sqrt(ab) * x0, beta[i - 1], ab, abp, v0hat=x0)
    assert np.allclose(vp0, np.sqrt(abp) * x0, rtol=0, atol=1e-12)


def test_last_step_returns_the_estimate_and_noise_enters_linearly():
    beta, abar = _schedule()
    rng = np.random.default_rng(0)
    v, v0, z = (rng.standard_normal((4, 6)) for _ in range(3))
    _, vp = oracle.ddpm_step(v, beta[0], abar[0], 1.0, v0hat=v0)
    assert np.allclose(vp, v0, rtol=0, atol=1e-12)
    _, a = oracle.ddpm_step(v, beta[99], abar[99], abar[98], v0hat=v0)
    _, b = oracle.ddpm_step(v, beta[99], abar[99], abar[98], v0hat=v0, z=z, sigma=0.3)
    assert np.allclose(b - a, 0.3 * z, rtol=0, atol=1e-12)
