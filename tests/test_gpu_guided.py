"""Judged surrogate-assisted guidance gradients (paper_2603_16393_amd.guided)
on the GPU: the prediction arithmetic, the judge's fallback and recovery
(forced from the host through its thresholds), and what the trained network
adds over reusing the last exact gradient."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2603_16393_amd", "weights", "surrogate_70x70.npy")
B = 4


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import fwi_inputs as fi
    from paper_2603_16393_amd import FwiPlan
    from paper_2603_16393_amd.surrogate import Surrogate, init_params

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    acq = fi.surface_acquisition(70, 70, ns=5, nt=1000, nb=40)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    plan = FwiPlan(acq, max_batch=B, device=dev)
    v_true = fi.faulted_model(70, 70, 1000)
    dobs = plan.forward(torch.tensor(v_true[None], dtype=torch.float32, device=dev), w, keep_for_adjoint=False)
    plan.set_obs(dobs[0].contiguous())
    sur = Surrogate(B, device=dev)
    sur.set_params(init_params(0, out_scale=0.016))
    zeta = torch.tensor(np.stack([fi.stand_in_zeta(70, 70, b) for b in range(B)]), dtype=torch.float32, device=dev)
    vt = torch.tensor(v_true, dtype=torch.float32, device=dev)
    return dev, plan, w, sur, zeta, vt


def _v(vt, zeta, t):
    return torch.clamp(vt + t * zeta, 1500.0, 4500.0).contiguous()


def test_mf_predict_arithmetic(setup):
    from paper_2603_16393_amd.surrogate import mf_predict

    dev = setup[0]
    g = torch.Generator(device=dev).manual_seed(0)
    a, s, sa = (torch.randn((3, 70, 70), device=dev, generator=g) for _ in range(3))
    Ja, Js, Jsa = (torch.rand(3, device=dev, dtype=torch.float64, generator=g) for _ in range(3))
    out = torch.empty_like(a)
    Jo = torch.empty_like(Ja)
    mf_predict(a, s, sa, out, Ja, Js, Jsa, Jo)
    assert torch.equal(out, a + (s - sa))
    assert torch.equal(Jo, Ja + (Js - Jsa))
    mf_predict(a, s, sa, a)  # in place on the anchor
    assert torch.equal(a, out)


def test_plain_below_switch_and_exact_values(setup):
    from paper_2603_16393_amd.guided import GuidanceGradients

    dev, plan, w, sur, zeta, vt = setup
    src = GuidanceGradients(plan, w, B, surrogate=sur, t_switch=0.5)
    v = _v(vt, zeta, 0.3)
    J, g = src(0.3, v)
    J, g = J.clone(), g.clone()
    d = plan.forward(v, w, keep_for_adjoint=True)
    J2, adj = plan.w2_misfit(d)
    g2 = plan.adjoint_gradient(v, adj)
    assert torch.equal(J, J2) and torch.equal(g, g2)
    assert src.stats.served_predicted == 0 and src.stats.surrogate_batches == 0


def test_judge_adapts_interval_and_falls_back(setup):
    """Always-pass thresholds double the interval; impossible ones drive it to 0
    (solver every step) while every returned gradient is the solver's."""
    from paper_2603_16393_amd.guided import GuidanceGradients

    dev, plan, w, sur, zeta, vt = setup
    ts = np.linspace(1.0, 0.6, 30)
    ok = GuidanceGradients(plan, w, B, surrogate=sur, cos_min=-2.0, jerr_max=1e30, k0=1, k_max=8)
    for t in ts:
        ok(float(t), _v(vt, zeta, float(t)))
    assert ok.stats.judged >= 2 and ok.stats.passed == ok.stats.judged
    assert max(ok.stats.k_trace) == 8
    assert ok.stats.served_predicted + ok.stats.served_exact == len(ts)
    assert ok.stats.served_predicted > len(ts) // 2

    bad = GuidanceGradients(plan, w, B, surrogate=sur, cos_min=1.5, jerr_max=-1.0, k0=4, k_max=8)
    for t in ts:
        J, g = bad(float(t), _v(vt, zeta, float(t)))
    assert bad.stats.passed == 0 and bad.stats.k_trace[-1] == 0
    # once the interval reached 0 every step is a judged solver step
    first_zero = bad.stats.k_trace.index(0)
    assert bad.stats.served_exact >= len(ts) - 8
    v = _v(vt, zeta, float(ts[-1]))
    d = plan.forward(v, w, keep_for_adjoint=True)
    J2, adj = plan.w2_misfit(d)
    assert torch.equal(J, J2)
    assert torch.equal(g, plan.adjoint_gradient(v, adj))
    assert first_zero <= 3


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained surrogate weights in the tree")
def test_trained_surrogate_improves_on_anchor_reuse(setup):
    """Same fixed schedule (judge every 8 steps over t in (1, 0.5]) with and
    without the trained network: the network's predictions of the misfit are
    closer to the solver's (measured with the 50,000-pair weights: median
    error 0.022 vs 0.042), and its gradients are no worse (judged cosine
    medians 0.988 vs 0.989).  The network does not improve the gradient
    itself, so on throughput it does not beat anchor reuse; this test holds it
    to the gain it does make."""
    from paper_2603_16393_amd.guided import GuidanceGradients
    from paper_2603_16393_amd.surrogate import Surrogate

    dev, plan, w, _, zeta, vt = setup
    net = Surrogate(B, device=dev)
    net.set_params(np.load(WEIGHTS))
    ts = np.linspace(1.0, 0.505, 100)
    res = {}
    for name, pred, s in (("net", "surrogate", net), ("anchor", "anchor", None)):
        src = GuidanceGradients(plan, w, B, surrogate=s, predictor=pred, k0=8, adapt=False,
                                cos_min=-2.0, jerr_max=1e30)
        for t in ts:
            src(float(t), _v(vt, zeta, float(t)))
        res[name] = (np.array(src.stats.judge_cos), np.array(src.stats.judge_jerr))
    net.close()
    cn, jn = res["net"]
    ca, ja = res["anchor"]
    print("judged cos median net / anchor", np.median(cn), np.median(ca), "misfit err median", np.median(jn),
          np.median(ja))
    assert np.median(jn) < 0.7 * np.median(ja)
    assert np.median(cn) >= np.median(ca) - 0.01


SCORE_WEIGHTS = os.path.join(ROOT, "paper_2603_16393_amd", "weights", "score_70x70.npy")


@pytest.mark.skipif(not (os.path.exists(WEIGHTS) and os.path.exists(SCORE_WEIGHTS)),
                    reason="no trained surrogate or score-network weights in the tree")
def test_trained_surrogate_gains_along_the_reverse_loop():
    """Along Algorithm 2's own trajectory (trained score network, guidance on, 100 respaced steps, 8 samples),
    the clean estimate moves far between steps at t > 0.5 (about 100 m/s RMS per step), so the gradient of
    the last solver step ages fast.  Four steps after an anchor, the network's multi-fidelity prediction
    g(v_a) + g_S(v) - g_S(v_a) is measurably closer to the solver's gradient than the anchor's gradient
    reused, and its misfit prediction is closer too.  Bars fixed before the run (the measured medians on 16
    samples were cosine 0.66 vs 0.39 and misfit error 0.043 vs 0.17): median cosine at least 0.1 higher and
    median misfit error at most half the anchor's.  Neither reaches the judge's 0.95 on this trajectory: there
    the solver runs every step."""
    from paper_2603_16393_amd import FwiPlan
    from paper_2603_16393_amd.diffusion import ReverseLoop
    from paper_2603_16393_amd.score import ScoreNet
    from paper_2603_16393_amd.surrogate import Surrogate

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import fwi_inputs as fi

    dev = torch.device("cuda:0")
    Bn, k = 8, 4
    acq = fi.surface_acquisition(70, 70, ns=5, nt=1000, nb=40)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    plan = FwiPlan(acq, max_batch=Bn, device=dev)
    vt = torch.tensor(fi.faulted_model(70, 70, 1000)[None], dtype=torch.float32, device=dev)
    plan.set_obs(plan.forward(vt, w, keep_for_adjoint=False)[0].contiguous())
    net = ScoreNet(Bn, device=dev)
    net.set_params(np.load(SCORE_WEIGHTS))
    sur = Surrogate(Bn, device=dev)
    sur.set_params(np.load(WEIGHTS))
    loop = ReverseLoop(net, Bn, 100, plan=plan, wavelet=w, guidance=dict(rho0=11.5))
    x = torch.tensor(np.random.default_rng(21).standard_normal((Bn, 70, 70)).astype(np.float32), device=dev)
    z = loop.step_noise(22)
    vs = []
    for s in range(len(loop.steps)):
        x.copy_(loop.step(x, s, z[s]))
        if loop.steps[s] / 1000.0 > 0.5:
            vs.append(loop.vphys.clone())
    ge, Je, gs, Js = [], [], [], []
    for v in vs:
        d = plan.forward(v, w, keep_for_adjoint=True)
        J, adj = plan.w2_misfit(d)
        ge.append(plan.adjoint_gradient(v, adj).double())
        Je.append(J.clone())
        ds = sur.forward(v)
        J2, adj2 = plan.w2_misfit(ds)
        gs.append(sur.backward(adj2).double())
        Js.append(J2.clone())
    torch.cuda.synchronize()

    def cos(a, b):
        a, b = a.reshape(Bn, -1), b.reshape(Bn, -1)
        return ((a * b).sum(1) / (a.norm(dim=1) * b.norm(dim=1))).cpu().numpy()

    ca, cs, ea, es = [], [], [], []
    for i in range(k, len(vs)):
        a = i - k
        ca.append(cos(ge[a], ge[i]))
        cs.append(cos(ge[a] + gs[i] - gs[a], ge[i]))
        ea.append((torch.abs(Je[a] - Je[i]) / Je[i]).cpu().numpy())
        es.append((torch.abs(Je[a] + Js[i] - Js[a] - Je[i]) / Je[i]).cpu().numpy())
    ca, cs, ea, es = (float(np.median(np.concatenate(q))) for q in (ca, cs, ea, es))
    print(f"reverse loop, {len(vs)} steps at t > 0.5, k = {k}: median cosine anchor {ca:.3f} network {cs:.3f}; "
          f"median misfit error anchor {ea:.3f} network {es:.3f}", flush=True)
    net.close()
    sur.close()
    plan.close()
    assert cs >= ca + 0.1
    assert es <= 0.5 * ea
