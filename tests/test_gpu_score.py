"""Score network on the GPU (BF16 matrix cores) vs its FP64 reference
(oracle/score.py with BF16 rounding where the GPU stores BF16), through the
C ABI: forward with the three output maps, the input VJP (the chain rule of
Eq. chain_rule for the clean estimate), every parameter group's gradient,
the denoising score-matching loss and gradient of a training step, bitwise
determinism, and a training run resumed from saved parameters and Adam state
equal to the uninterrupted one.

Bars come from the reference's own sensitivity: perturbing x by 1e-7
relative flips BF16 roundings at about the rate FP32 accumulation order does,
and the resulting change of the reference output (or gradient) times 4 is
the bar (with a floor), computed in each test.
"""
import numpy as np
import pytest

import fwi_inputs as fi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

B = 3
T = np.array([0.05, 0.5, 0.93])


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


@pytest.fixture(scope="module")
def setup(dev):
    from oracle import score as S
    from paper_2603_16393_amd.score import ScoreNet, output_map, vp_schedule

    p = S.init_params(11)
    rng = np.random.default_rng(12)
    for n in p:
        if p[n].ndim == 1:
            p[n] = 0.1 * rng.standard_normal(p[n].shape)
    vec = S.pack(p).astype(np.float32)
    p32 = S.unpack(vec.astype(np.float64))            # the FP32 parameters both sides use
    x0 = np.stack([fi.to_normalised(fi.faulted_model(70, 70, s)) for s in range(B)])
    _, abar = vp_schedule()
    ab = abar[(T * 1000).astype(int) - 1]
    noise = rng.standard_normal(x0.shape)
    x = (np.sqrt(ab)[:, None, None] * x0 + np.sqrt(1 - ab)[:, None, None] * noise).astype(np.float32)
    net = ScoreNet(B, device=dev)
    net.set_params(vec)
    yield dict(S=S, p=p32, vec=vec, x=x.astype(np.float64), x32=x, ab=ab, net=net, output_map=output_map,
               rng=rng)
    net.close()


def _t(a, dev):
    return torch.tensor(np.ascontiguousarray(a, np.float32), device=dev)


def _sens(S, p, x, t, skip, scale, a):
    """Change of the reference output and VJP under a 1e-7 relative perturbation of x."""
    rng = np.random.default_rng(99)
    xp = x * (1 + 1e-7 * rng.standard_normal(x.shape))
    o0, c0 = S.forward(p, x, t, skip, scale)
    o1, c1 = S.forward(p, xp, t, skip, scale)
    d0, g0 = S.backward(p, c0, a)
    d1, g1 = S.backward(p, c1, a)
    return o0, c0, d0, g0, _rel(o1, o0), _rel(d1, d0), {n: _rel(g1[n], g0[n]) for n in g0}


@pytest.mark.parametrize("kind", ["eps", "score", "clean"])
def test_forward_and_vjp_match_reference(setup, dev, kind):
    S, p, net = setup["S"], setup["p"], setup["net"]
    skip, scale = setup["output_map"](kind, setup["ab"])
    skip32, scale32 = skip.astype(np.float32), scale.astype(np.float32)
    a = np.random.default_rng(5).standard_normal(setup["x"].shape).astype(np.float32)
    o_ref, _, dx_ref, g_ref, s_o, s_d, s_g = _sens(S, p, setup["x"], T, skip32.astype(np.float64),
                                                   scale32.astype(np.float64), a.astype(np.float64))
    out = net.forward(_t(setup["x32"], dev), _t(T, dev), _t(skip32, dev), _t(scale32, dev))
    dx = net.backward(_t(a, dev), weight_grads=True)
    torch.cuda.synchronize()
    G = S.unpack(net.get_grads().astype(np.float64))
    e_o = _rel(out.cpu().numpy(), o_ref)
    e_d = _rel(dx.cpu().numpy(), dx_ref)
    bar_o, bar_d = max(4 * s_o, 2e-3), max(4 * s_d, 5e-3)
    print(f"score {kind}: out {e_o:.2e} (bar {bar_o:.1e}), dx {e_d:.2e} (bar {bar_d:.1e})", flush=True)
    assert e_o <= bar_o
    assert e_d <= bar_d
    worst = []
    for n in g_ref:
        e = _rel(G[n], g_ref[n])
        bar = max(4 * s_g[n], 1e-2)
        worst.append((e / bar, n, e, bar))
        assert e <= bar, (n, e, bar)
    print("  worst parameter groups (err / bar):", sorted(worst)[-3:], flush=True)


def test_deterministic(setup, dev):
    net = setup["net"]
    x, t = _t(setup["x32"], dev), _t(T, dev)
    a = _t(np.random.default_rng(6).standard_normal(setup["x"].shape), dev)
    o1 = net.forward(x, t).clone()
    d1 = net.backward(a, weight_grads=True).clone()
    g1 = net.get_grads()
    o2 = net.forward(x, t)
    d2 = net.backward(a, weight_grads=True)
    g2 = net.get_grads()
    assert torch.equal(o1, o2) and torch.equal(d1, d2) and np.array_equal(g1, g2)


def test_backward_needs_the_same_batch(setup, dev):
    from paper_2603_16393_amd import _lib

    net = setup["net"]
    net.forward(_t(setup["x32"], dev), _t(T, dev))
    with pytest.raises(_lib.FwiError) as e:
        net.backward(_t(np.zeros((2, 70, 70)), dev))
    assert e.value.code == _lib.FWI_ESTATE


def test_train_step_loss_and_gradient(setup, dev):
    S, p, net = setup["S"], setup["p"], setup["net"]
    from paper_2603_16393_amd.score import vp_schedule

    _, abar = vp_schedule()
    rng = np.random.default_rng(21)
    x0 = np.stack([fi.to_normalised(fi.faulted_model(70, 70, 40 + s)) for s in range(B)]).astype(np.float32)
    noise = rng.standard_normal(x0.shape).astype(np.float32)
    ti = np.array([30, 480, 990])
    ab = abar[ti - 1]
    sa, s1a = np.sqrt(ab).astype(np.float32), np.sqrt(1 - ab).astype(np.float32)
    # the reference on the FP32 noised state the GPU forms (x_t = fma(sa, x0, s1a noise) in FP32)
    xt = (sa.astype(np.float32)[:, None, None] * x0 + s1a[:, None, None] * noise).astype(np.float32)
    eps, cache = S.forward(p, xt.astype(np.float64), ti / 1000.0)
    r = eps - noise
    loss_ref = float(np.mean(r * r))
    _, g_ref = S.backward(p, cache, 2 * r / r.size)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    net.set_params(setup["vec"])
    net.train_step(_t(x0, dev), _t(noise, dev), _t(ti / 1000.0, dev), _t(sa, dev), _t(s1a, dev), lr=1e-4,
                   loss_out=loss)
    torch.cuda.synchronize()
    G = S.unpack(net.get_grads().astype(np.float64))
    net.set_params(setup["vec"])   # restore for the other tests
    e_l = abs(float(loss.item()) - loss_ref) / loss_ref
    print(f"score DSM loss {loss.item():.6f} vs {loss_ref:.6f} (rel {e_l:.1e})", flush=True)
    assert e_l <= 2e-3
    for n in g_ref:
        assert _rel(G[n], g_ref[n]) <= 5e-2, (n, _rel(G[n], g_ref[n]))


def test_resumed_training_equals_uninterrupted(setup, dev):
    from paper_2603_16393_amd.score import ScoreNet, vp_schedule

    _, abar = vp_schedule()
    rng = np.random.default_rng(31)
    batches = []
    for k in range(5):
        x0 = np.stack([fi.to_normalised(fi.faulted_model(70, 70, 100 + 3 * k + s)) for s in range(B)])
        ti = rng.integers(1, 1001, B)
        ab = abar[ti - 1]
        batches.append([_t(a, dev) for a in (x0, rng.standard_normal(x0.shape), ti / 1000.0, np.sqrt(ab),
                                             np.sqrt(1 - ab))])
    a = ScoreNet(B, device=dev)
    a.set_params(setup["vec"])
    for bt in batches[:3]:
        a.train_step(*bt, lr=3e-4)
    saved = (a.get_params(), *a.get_adam())
    for bt in batches[3:]:
        a.train_step(*bt, lr=3e-4)
    final_a = a.get_params()
    b = ScoreNet(B, device=dev)
    b.set_params(saved[0])
    b.set_adam(saved[1], saved[2], saved[3])
    assert saved[3] == 3
    for bt in batches[3:]:
        b.train_step(*bt, lr=3e-4)
    final_b = b.get_params()
    assert np.array_equal(final_a, final_b)
    assert not np.array_equal(final_a, saved[0])
    a.close()
    b.close()
