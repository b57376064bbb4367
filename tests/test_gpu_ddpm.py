"""Reverse DDPM step (Algorithm 2 before its guidance term) on the GPU vs the
FP64 oracle, through the C ABI: the clean estimator from a score and the
posterior mean plus noise, with the estimate given instead of the score, with
and without noise, on the batch's 16 x 70 x 70 layout and a ragged length
(float4 body and scalar tail).  Bar: 2e-6 relative to the largest value
(FP32 elementwise, a few roundings).  A reverse chain of 100 steps under the
exact score of a point-mass prior (its clean estimate is that point at every
step) with sigma = 0 must end at that point.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _schedule(N=1000):
    beta = np.linspace(1e-4, 0.02, N)
    return beta, np.cumprod(1.0 - beta)


@pytest.mark.parametrize("shape", [(16, 70, 70), (3, 7, 5)])
@pytest.mark.parametrize("mode", ["score", "estimate", "score_noise"])
def test_ddpm_step_matches_oracle(dev, shape, mode):
    import oracle
    from paper_2603_16393_amd import ddpm_step

    beta, abar = _schedule()
    rng = np.random.default_rng(len(shape) * 7 + len(mode))
    v, s, z = (rng.standard_normal(shape).astype(np.float32) for _ in range(3))
    x0 = (2.0 * rng.standard_normal(shape)).astype(np.float32)
    i = 400
    kw = dict(beta=beta[i - 1], abar=abar[i - 1], abar_prev=abar[i - 2])
    t = lambda a: torch.tensor(a, device=dev)  # noqa: E731
    if mode == "estimate":
        x_o, vp_o = oracle.ddpm_step(v, v0hat=x0, **kw)
        x_g, vp_g = ddpm_step(t(v), v0hat=t(x0), **kw)
    else:
        sig = 0.7 if mode == "score_noise" else 0.0
        x_o, vp_o = oracle.ddpm_step(v, score=s, z=z if sig else None, sigma=sig, **kw)
        x_g, vp_g = ddpm_step(t(v), score=t(s), z=t(z) if sig else None, sigma=sig, **kw)
    torch.cuda.synchronize()
    for g_, o_ in ((x_g, x_o), (vp_g, vp_o)):
        err = np.abs(g_.cpu().numpy() - o_).max() / np.abs(o_).max()
        assert err <= 2e-6, err


def test_reverse_chain_reaches_the_point_mass(dev):
    from paper_2603_16393_amd import ddpm_step

    beta, abar = _schedule(100)
    rng = np.random.default_rng(3)
    xs = torch.tensor(rng.uniform(-1, 1, (4, 70, 70)).astype(np.float32), device=dev)
    v = torch.tensor(rng.standard_normal((4, 70, 70)).astype(np.float32), device=dev)
    for i in range(100, 0, -1):
        ab, abp = abar[i - 1], (abar[i - 2] if i > 1 else 1.0)
        score = -(v - float(np.sqrt(ab)) * xs) / float(1.0 - ab)
        _, v = ddpm_step(v, float(beta[i - 1]), float(ab), float(abp), score=score.contiguous())
    torch.cuda.synchronize()
    assert float((v - xs).abs().max()) <= 1e-4
