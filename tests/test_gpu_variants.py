"""Comparison and ablation variants of the guidance (Sec. 4 Algorithm 1, Sec. 6)
on the GPU, through the C ABI, against the FP64 oracle.

* fwi_l2_misfit on identical FP32 traces: FP64 sums on both sides, so J agrees
  to 1e-10 relative and the adjoint source to FP32 rounding (rel L2 <= 1e-7).
* fwi_tv_subgradient: the signs are exact on both sides, so every entry agrees
  to FP32 rounding of g + alpha q.
* Whole steps (forward, misfit, adjoint gradient, update) of baseline DPS with
  the least-squares potential, its enhanced ablation form, and the W2+TV and
  OT-WE+TV descent baselines: gradients to the path's 1e-4 relative L2 bar,
  misfits to 1e-5; the update to 1e-4, or, with the diagonal preconditioner,
  to the bar that the preconditioner's sensitivity to a gradient error at the
  1e-4 level implies (measured on the oracle alone).
Every oracle input is the FP32 array the GPU receives, or oracle output.
"""
import sys

import numpy as np
import pytest

import fwi_inputs as fi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.linalg.norm(b))


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def _t(x, dev, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _traces(seed, shape):
    rng = np.random.default_rng(seed)
    t = np.arange(shape[-1])
    env = np.exp(-0.5 * ((t - shape[-1] / 3) / (shape[-1] / 10)) ** 2)
    return (rng.standard_normal(shape) * env).astype(np.float32)


L2_CASES = [dict(sigma=0.05, k=0.0, normalize=False), dict(sigma=0.05, k=100.0, normalize=False),
            dict(sigma=1.0, k=100.0, normalize=True), dict(sigma=1.0, k=0.0, normalize=True),
            dict(sigma=0.3, k=3.0, normalize=True)]


@pytest.mark.parametrize("shape", [(3, 2, 7, 301), (16, 5, 70, 1000)])
def test_l2_misfit_identical_inputs(dev, shape):
    import oracle
    from paper_2603_16393_amd import FwiPlan

    B, ns, nr, nt = shape
    acq = fi.surface_acquisition(70, 70, ns=ns, nt=nt, nb=10, rec_cols=np.arange(nr))
    plan = FwiPlan(acq, max_batch=B, device=dev)
    d_obs = _traces(1, (ns, nr, nt))
    d_syn = (d_obs[None] + 0.3 * np.stack([_traces(10 + b, (ns, nr, nt)) for b in range(B)])).astype(np.float32)
    for kw in L2_CASES:
        J, adj = plan.l2_misfit(_t(d_syn, dev), _t(d_obs, dev), **kw)
        J, adj = J.cpu().numpy(), adj.cpu().numpy()
        Jo, adjo = oracle.l2_misfit(_f32(d_syn), _f32(d_obs), **kw)
        eJ = float(np.max(np.abs(J - Jo) / np.abs(Jo)))
        ea = _rel(adj, adjo)
        _say(f"l2 {shape} {kw}: J rel {eJ:.1e}, adjoint rel L2 {ea:.1e}")
        assert eJ <= 1e-10 and ea <= 1e-7, kw
        assert np.max(np.abs(adj - adjo)) <= 2e-7 * np.max(np.abs(adjo))
    # J only (no adjoint source requested) gives the same J, bit for bit
    J1, _ = plan.l2_misfit(_t(d_syn, dev), _t(d_obs, dev), k=100.0, normalize=True)
    J2, a2 = plan.l2_misfit(_t(d_syn, dev), _t(d_obs, dev), k=100.0, normalize=True, want_adjoint=False)
    assert a2 is None and torch.equal(J1, J2)
    plan.close()


def test_l2_misfit_degenerate_cases(dev):
    import oracle
    from paper_2603_16393_amd import FwiPlan, _lib

    acq = fi.surface_acquisition(30, 30, ns=2, nt=64, nb=5)
    plan = FwiPlan(acq, max_batch=2, device=dev)
    shape = (acq.ns, acq.nr, acq.nt)
    zero = np.zeros(shape, np.float32)
    d = np.full((2,) + shape, 0.25, np.float32)
    for kw in (dict(k=100.0, normalize=True), dict(sigma=0.5)):
        J, adj = plan.l2_misfit(_t(d, dev), _t(zero, dev), **kw)
        Jo, adjo = oracle.l2_misfit(_f32(d), _f32(zero), **kw)
        assert np.allclose(J.cpu().numpy(), Jo, rtol=1e-12) and np.allclose(adj.cpu().numpy(), adjo, rtol=1e-7)
    J, adj = plan.l2_misfit(_t(d[:1], dev), _t(d[0], dev), k=100.0, normalize=True)
    assert float(J[0]) == 0.0 and not torch.any(adj)
    # argument errors
    for kw in (dict(sigma=0.0), dict(k=-1.0), dict(sigma=float("nan"))):
        with pytest.raises(_lib.FwiError):
            plan.l2_misfit(_t(d, dev), _t(zero, dev), **kw)
    plan.close()


def _tv_fields():
    rng = np.random.default_rng(5)
    lay = fi.layered_model(70, 70, 3)                     # piecewise constant: ties everywhere
    flt = fi.faulted_model(70, 70, 4)
    yield "layered+faulted", np.stack([lay, flt]).astype(np.float32)
    yield "random 23x37", rng.standard_normal((3, 23, 37)).astype(np.float32)
    yield "integers", np.round(rng.standard_normal((2, 9, 9)) * 2).astype(np.float32)
    yield "1x8", rng.standard_normal((1, 1, 8)).astype(np.float32)
    yield "5x1", rng.standard_normal((2, 5, 1)).astype(np.float32)
    yield "1x1", rng.standard_normal((1, 1, 1)).astype(np.float32)


@pytest.mark.parametrize("name,x", list(_tv_fields()))
def test_tv_subgradient(dev, name, x):
    import oracle
    from paper_2603_16393_amd import tv_subgradient

    B, nz, nx = x.shape
    g = (np.random.default_rng(2).standard_normal(x.shape) * 1e-3).astype(np.float32)
    for alpha, with_g in ((1.0, False), (0.37, True), (-2.0, True)):
        xg = _t(x, dev)
        gg = _t(g, dev) if with_g else None
        out = tv_subgradient(xg, gg, alpha).cpu().numpy()
        ref = oracle.tv_subgradient(_f32(x), _f32(g) if with_g else None, alpha)
        tol = 1e-6 * (np.max(np.abs(g)) * with_g + abs(alpha) * 4.0 / (nz * nx))
        assert np.max(np.abs(out - ref)) <= tol, (name, alpha, with_g)
    # in place on g
    gg = _t(g, dev)
    tv_subgradient(_t(x, dev), gg, 0.5, out=gg)
    ref = oracle.tv_subgradient(_f32(x), _f32(g), 0.5)
    assert np.max(np.abs(gg.cpu().numpy() - ref)) <= 1e-6 * (np.max(np.abs(g)) + 2.0 / (nz * nx))


def test_tv_subgradient_argument_errors(dev):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    x = _t(np.zeros((1, 4, 4), np.float32), dev)
    p = lambda t: __import__("ctypes").c_void_p(t.data_ptr())
    assert L.fwi_tv_subgradient(1, 4, 4, p(x), None, 1.0, p(x), None) == -1      # out aliases v
    assert L.fwi_tv_subgradient(1, 0, 4, p(x), None, 1.0, p(x), None) == -1
    assert L.fwi_tv_subgradient(0, 4, 4, None, None, 1.0, None, None) == 0


def _setup(dev, seed=11):
    """Ragged grid, 3 shots on the surface, two samples near a faulted truth."""
    acq = fi.surface_acquisition(23, 37, ns=3, nt=350, nb=5, rec_cols=np.arange(1, 37, 2))
    vt = fi.faulted_model(23, 37, seed)
    v = np.clip(np.stack([vt * (1 + 0.04 * np.sin(np.arange(37) / (3.0 + b))[None, :]) for b in range(2)]),
                1500, 4500).astype(np.float32)
    w = fi.ricker(acq.nt, acq.dt, acq.f_peak).astype(np.float32)
    return acq, v, vt.astype(np.float32), w


@pytest.mark.parametrize("kw", [dict(sigma=0.05, k=0.0, normalize=False), dict(sigma=1.0, k=100.0, normalize=True)])
def test_dps_least_squares_step(dev, kw):
    """Baseline DPS (Algorithm 1) with Phi_l2, and its enhanced ablation form:
    forward, least-squares misfit, adjoint gradient, scalar step zeta g."""
    import oracle
    from paper_2603_16393_amd import FwiPlan, guidance_step

    acq, v, vt, w = _setup(dev)
    d_obs = oracle.forward(acq, _f32(vt), _f32(w)).astype(np.float32)
    plan = FwiPlan(acq, max_batch=2, device=dev)
    vg, wt = _t(v, dev), _t(w, dev)
    d = plan.forward(vg, wt, keep_for_adjoint=True)
    J, adj = plan.l2_misfit(d, _t(d_obs, dev), **kw)
    g = plan.adjoint_gradient(vg, adj)
    zeta = 30.0 / float(g.abs().max())  # largest update 30 m/s
    vn, _ = guidance_step(vg, g, g, vg, rho0=zeta, gamma=0.0, tau=1e30)
    torch.cuda.synchronize()
    assert plan.status() == 0
    d_o = oracle.forward(acq, _f32(v), _f32(w))
    Jo, adjo = oracle.l2_misfit(d_o, _f32(d_obs), **kw)
    go = oracle.gradient(acq, _f32(v), _f32(w), adjo)
    vno, _, _, _ = oracle.guidance(_f32(v), go, go, _f32(v), rho0=zeta, gamma=0.0, tau=1e30)
    eJ = float(np.max(np.abs(J.cpu().numpy() - Jo) / np.abs(Jo)))
    eg = _rel(g.cpu().numpy(), go)
    ev = _rel(vn.cpu().numpy() - _f32(v), vno - _f32(v))
    _say(f"DPS l2 step {kw}: J rel {eJ:.2e}, grad rel L2 {eg:.2e}, update rel L2 {ev:.2e}")
    assert eJ <= 1e-5 and eg <= 1e-4 and ev <= 1e-4
    plan.close()


@pytest.mark.parametrize("name,w2kw,stepkw", [
    ("W2+TV", dict(k=0.0, squared=True), dict(gamma=0.0, tau=1e30)),
    ("OT-WE+TV", dict(k=100.0), dict(gamma=0.55, c=0.1, tau=0.0)),
])
def test_tv_descent_baseline_step(dev, name, w2kw, stepkw):
    """v <- v - P(v) (grad J + alpha g_TV(v)) with P = rho0 (W2+TV, raw-trace
    squared W2) or rho(v) D(v) (OT-WE+TV, the enhanced W2)."""
    import oracle
    from paper_2603_16393_amd import FwiPlan, guidance_step, tv_subgradient

    acq, v, vt, w = _setup(dev, 13)
    d_obs = oracle.forward(acq, _f32(vt), _f32(w)).astype(np.float32)
    plan = FwiPlan(acq, max_batch=2, device=dev)
    plan.set_obs(_t(d_obs, dev), **w2kw)
    vg, wt = _t(v, dev), _t(w, dev)
    d = plan.forward(vg, wt, keep_for_adjoint=True)
    J, adj = plan.w2_misfit(d)
    g = plan.adjoint_gradient(vg, adj)
    # the TV term's entries reach 0.4 max|g|; the step acts on the model in the diffusion state's units
    # x = v / 1500 - 2 (dJ/dx = 1500 dJ/dv), largest update 0.05
    alpha = 0.1 * float(g.abs().max()) * v.shape[1] * v.shape[2]
    h = tv_subgradient(vg, g, alpha)
    x = fi.to_normalised(v).astype(np.float32)
    xg = _t(x, dev)
    rho0 = 0.05 / (1500.0 * float(h.abs().max()))
    xn, _ = guidance_step(xg, h, g, xg, rho0=rho0, unit_scale=1500.0, **stepkw)
    torch.cuda.synchronize()
    assert plan.status() == 0
    obs = oracle.w2_prepare(_f32(d_obs), acq.dt, k=w2kw["k"], squared=w2kw.get("squared", False))
    Jo, go, _, _ = oracle.objective_and_gradient(acq, _f32(v), _f32(w), obs)
    ho = oracle.tv_subgradient(_f32(v), go, alpha)
    xno, _, _, _ = oracle.guidance(_f32(x), ho, go, _f32(x), rho0=rho0, unit_scale=1500.0, **stepkw)
    eJ = float(np.max(np.abs(J.cpu().numpy() - Jo) / np.abs(Jo)))
    eg, eh = _rel(g.cpu().numpy(), go), _rel(h.cpu().numpy(), ho)
    ev = _rel(xn.cpu().numpy() - _f32(x), xno - _f32(x))
    # The update's bar follows from the gradient's: kappa = ((max|g| + eps)/(|g_j| + eps))^gamma turns a
    # pointwise gradient error into gamma times its relative size, largest where g is small and the TV
    # term keeps h large.  Perturb the oracle's gradient by FP32-like absolute noise at the 1e-4 bar
    # (oracle only) and allow 3x the worst resulting change of the update.
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(4):
        gp = go + 1e-4 * np.sqrt(np.mean(go ** 2)) * rng.standard_normal(go.shape)
        xp, _, _, _ = oracle.guidance(_f32(x), oracle.tv_subgradient(_f32(v), gp, alpha), gp, _f32(x), rho0=rho0,
                                      unit_scale=1500.0, **stepkw)
        worst = max(worst, _rel(xp - _f32(x), xno - _f32(x)))
    bar = max(1e-4, 3.0 * worst)
    _say(f"{name} step: J rel {eJ:.2e}, grad rel L2 {eg:.2e}, g + alpha g_TV rel L2 {eh:.2e}, "
         f"update rel L2 {ev:.2e} (bar {bar:.1e})")
    assert eJ <= 1e-5 and eg <= 1e-4 and eh <= 1e-4 and ev <= bar
    plan.close()
