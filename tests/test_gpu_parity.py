"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Bars (written in each test): relative L2 <= 1e-4 on seismograms and
gradients, <= 1e-5 relative on W2 misfit values (the FP32-stencil targets);
the W2 stage and the guidance update alone, on identical inputs, are held
far tighter.  Inputs are seeded synthetic models; every oracle input is the
same FP32-rounded array the GPU receives.
"""
import dataclasses
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


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_16393_amd import _lib

    _lib.load()
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _t(x, dev, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------------------
# configurations
def _config0():
    """One shot at the surface centre, 70x70 three-layer model, 40-cell sponge."""
    acq = fi.surface_acquisition(70, 70, ns=1, shot_cols=[35], nt=1000, nb=40)
    v = fi.layered_model(70, 70, 0)
    vt = fi.blob_perturbation(v, 1)
    return acq, v[None], vt


def _small(seed, nz=23, nx=37, nb=5, fs=True, ns=3, nt=350, one_row=None):
    """Ragged grid.  one_row=None: a sparse surface spread plus interior
    receivers (tiled path only); one_row=k: every other column of row k (the
    LDS-resident path needs all receivers on one row)."""
    rng = np.random.default_rng(seed)
    acq = fi.surface_acquisition(nz, nx, ns=ns, nt=nt, nb=nb, free_surface=fs)
    if one_row is None:
        acq.rec_iz = np.concatenate([np.zeros(nx // 2, np.int32), rng.integers(1, nz, 4).astype(np.int32)])
        acq.rec_ix = np.concatenate([np.arange(0, nx, 2, dtype=np.int32)[: nx // 2],
                                     rng.integers(0, nx, 4).astype(np.int32)])
        # receivers must be distinct nodes
        _, keep = np.unique(acq.rec_iz.astype(np.int64) * 1000 + acq.rec_ix, return_index=True)
        acq.rec_iz, acq.rec_ix = acq.rec_iz[np.sort(keep)], acq.rec_ix[np.sort(keep)]
    else:
        acq.rec_ix = np.arange(1, nx, 2, dtype=np.int32)
        acq.rec_iz = np.full(len(acq.rec_ix), one_row, np.int32)
    vt = fi.faulted_model(nz, nx, seed)
    v = np.stack([vt * (1 + 0.04 * np.sin(np.arange(nx) / (3.0 + b))[None, :]) for b in range(2)])
    v = np.clip(v, 1500, 4500)
    return acq, v, vt


def _oracle_obs(acq, vt):
    """Observations from the true model by the oracle (FP32-rounded), given to both sides."""
    import oracle

    w = fi.ricker(acq.nt, acq.dt, acq.f_peak)
    return oracle.forward(acq, _f32(vt[None]), _f32(w))[0].astype(np.float32)


def _run_gpu(acq, v, vt, dev, force_path=-1, ckpt_every=0, budget=0, dobs=None):
    """dobs: the observations (the oracle's for gradient parity); None models them on the GPU."""
    from paper_2603_16393_amd import FwiPlan

    w = fi.ricker(acq.nt, acq.dt, acq.f_peak)
    B = v.shape[0]
    plan = FwiPlan(acq, max_batch=B, device=dev, force_path=force_path, ckpt_every=ckpt_every,
                   mem_budget_bytes=budget)
    wt = _t(w, dev)
    if dobs is None:
        dobs = plan.forward(_t(vt[None], dev), wt, keep_for_adjoint=False)[0].contiguous()
    else:
        dobs = _t(dobs, dev)
    plan.set_obs(dobs)
    vg = _t(v, dev)
    d = plan.forward(vg, wt, keep_for_adjoint=True)
    J, adj = plan.w2_misfit(d)
    g = plan.adjoint_gradient(vg, adj)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = dict(dobs=dobs.cpu().numpy(), d=d.cpu().numpy(), J=J.cpu().numpy(), adj=adj.cpu().numpy(),
               g=g.cpu().numpy(), info=plan.info, w=w)
    plan.close()
    return out


def _run_oracle(acq, v, dobs, w):
    import oracle

    obs = oracle.w2_prepare(_f32(dobs), acq.dt)
    J, g, d, adj = oracle.objective_and_gradient(acq, _f32(v), _f32(w), obs)
    return dict(J=J, g=g, d=d, adj=adj, obs=obs)


# ---------------------------------------------------------------------------
def test_forward_traces_config0(dev):
    import oracle

    acq, v, vt = _config0()
    r = _run_gpu(acq, v, vt, dev)
    assert r["info"]["path"] == 0
    d_o = oracle.forward(acq, _f32(v), _f32(r["w"]))
    dobs_o = oracle.forward(acq, _f32(vt[None]), _f32(r["w"]))[0]
    e1, e2 = _rel(r["d"], d_o), _rel(r["dobs"], dobs_o)
    _say(f"forward config0 (70x70, 1 shot, 1000 steps): traces rel L2 {e1:.2e} / {e2:.2e}")
    assert e1 <= 1e-4
    assert e2 <= 1e-4
    assert np.all(r["d"][..., 0] == 0.0)


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("fs", [True, False])
def test_forward_traces_ragged(dev, path, fs):
    """Ragged grid (23 x 37 + sponge: partial tiles and strips), interior
    receivers, both execution paths, reflecting and absorbing top."""
    import oracle

    acq, v, vt = _small(7, fs=fs, one_row=(3 if path == 0 else None))
    r = _run_gpu(acq, v, vt, dev, force_path=path)
    assert r["info"]["path"] == path
    d_o = oracle.forward(acq, _f32(v), _f32(r["w"]))
    e = _rel(r["d"], d_o)
    _say(f"forward ragged path={path} fs={fs}: traces rel L2 {e:.2e}")
    assert e <= 1e-4


def test_w2_stage_identical_inputs(dev):
    """Misfit and adjoint source on the very same FP32 traces: FP64 on both
    sides, so J agrees to 1e-10 and the adjoint source to 1e-7."""
    import oracle
    from paper_2603_16393_amd import FwiPlan

    acq, v, vt = _small(3, nt=500)
    rng = np.random.default_rng(0)
    w = fi.ricker(acq.nt, acq.dt, acq.f_peak)
    dobs = oracle.forward(acq, vt, w).astype(np.float32)
    dsyn = (oracle.forward(acq, v, w) + 1e-4 * rng.standard_normal((v.shape[0],) + dobs.shape)).astype(np.float32)
    for squared, reduction, k in [(False, 0, 100.0), (True, 0, 0.0), (False, 1, 100.0)]:
        plan = FwiPlan(acq, max_batch=v.shape[0], device=dev)
        plan.set_obs(_t(dobs, dev), k=k, squared=squared, reduction=reduction)
        J, adj = plan.w2_misfit(_t(dsyn, dev))
        J, adj = J.cpu().numpy(), adj.cpu().numpy()
        obs = oracle.w2_prepare(_f32(dobs), acq.dt, k=k, squared=squared)
        Jo, adjo, _ = oracle.w2_misfit(obs, _f32(dsyn), reduction=reduction)
        assert np.max(np.abs(J - Jo) / np.abs(Jo)) <= 1e-10, (squared, reduction)
        assert _rel(adj, adjo) <= 1e-7, (squared, reduction)
        plan.close()


def test_gradient_config0(dev):
    """Full chain on the one-shot configuration: J to 1e-5, dJ/dv to 1e-4."""
    acq, v, vt = _config0()
    dobs = _oracle_obs(acq, vt)
    r = _run_gpu(acq, v, vt, dev, dobs=dobs)
    o = _run_oracle(acq, v, dobs, r["w"])
    eJ = abs(r["J"][0] - o["J"][0]) / abs(o["J"][0])
    eg = _rel(r["g"], o["g"])
    ea = _rel(r["adj"], o["adj"])
    _say(f"gradient config0: J rel {eJ:.2e}, adjoint source rel L2 {ea:.2e}, grad rel L2 {eg:.2e}")
    assert eJ <= 1e-5
    assert eg <= 1e-4


@pytest.mark.parametrize("path,ckpt", [(0, 0), (1, 0), (1, 7), (1, 349)])
def test_gradient_ragged_paths(dev, path, ckpt):
    """Ragged grid, interior receivers, two samples: LDS-resident, tiled with
    the full history, tiled with checkpoints every 7 steps (ragged last
    segment) and with a single segment."""
    acq, v, vt = _small(11, one_row=(0 if path == 0 else None))
    dobs = _oracle_obs(acq, vt)
    r = _run_gpu(acq, v, vt, dev, force_path=path, ckpt_every=ckpt, dobs=dobs)
    assert r["info"]["path"] == path and r["info"]["store_mode"] == (1 if ckpt else 0)
    o = _run_oracle(acq, v, dobs, r["w"])
    eJ = np.max(np.abs(r["J"] - o["J"]) / np.abs(o["J"]))
    eg = _rel(r["g"], o["g"])
    _say(f"gradient ragged path={path} ckpt={ckpt}: J rel {eJ:.2e}, grad rel L2 {eg:.2e}")
    assert eJ <= 1e-5
    assert eg <= 1e-4


def test_guidance_step_parity(dev):
    import oracle
    from paper_2603_16393_amd import guidance_step

    rng = np.random.default_rng(1)
    B, nz, nx = 4, 70, 70
    vp, h, g = (rng.standard_normal((B, nz, nx)).astype(np.float32) for _ in range(3))
    x0 = np.stack([fi.to_normalised(fi.faulted_model(nz, nx, s)) for s in range(B)]).astype(np.float32)
    g *= 1e-6
    h *= 1e-6
    for kw in [dict(), dict(gamma=0.0, tau=1e9, rho0=0.3), dict(kappa_max=4.0, gamma=0.35, rho0=12.4, tau=0.02)]:
        vn, rho = guidance_step(_t(vp, dev), _t(h, dev), _t(g, dev), _t(x0, dev), unit_scale=1500.0, **kw)
        vn_o, rho_o, _, _ = oracle.guidance(_f32(vp), _f32(h), _f32(g), _f32(x0), unit_scale=1500.0, **kw)
        assert _rel(vn.cpu().numpy(), vn_o) <= 1e-6
        assert np.allclose(rho.cpu().numpy(), rho_o, rtol=1e-6)


def test_invalid_velocity_flag(dev):
    """A velocity above v_max is reported by the device flag, not a fault."""
    from paper_2603_16393_amd import FwiPlan

    acq = fi.surface_acquisition(20, 20, ns=1, nt=50, nb=4)
    plan = FwiPlan(acq, max_batch=1, device=dev)
    v = np.full((1, 20, 20), 2000.0)
    v[0, 3, 3] = 9000.0
    plan.forward(_t(v, dev), _t(fi.ricker(50, acq.dt, 15.0), dev), keep_for_adjoint=False)
    assert plan.status() == -6
    assert plan.status() == 0
    plan.close()


def test_bitwise_deterministic(dev):
    acq, v, vt = _small(5)
    a = _run_gpu(acq, v, vt, dev)
    b = _run_gpu(acq, v, vt, dev)
    for k in ("d", "J", "adj", "g"):
        assert np.array_equal(a[k], b[k]), k
