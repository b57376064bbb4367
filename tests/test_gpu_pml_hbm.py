"""PML swept from HBM (plan path 3): fields too large for the LDS-resident PML
sweeps, a forward history that does not fit, and checkpointed gradients
(Sec. 2.1 absorbing boundary realised by a PML; Sec. 6.1: 6 grid points on the
left, right and bottom, reflecting top).

* Each cell undergoes the LDS-resident sweep's operations in the same order, so
  on grids both paths take the traces and gradients are equal bit for bit, also
  with checkpoints (ragged intervals) and on three calls in a row.
* A field wider than the row bands can hold (the bottom layer of one band
  exceeds a workgroup's cells), picked automatically: oracle parity of the
  traces (1e-4 relative L2), J (1e-5) and the gradient (1e-4), full history and
  checkpointed.
* Full size, 400 x 800 with 4000 steps and 2 of the 20 shots: the checkpointed
  gradient equals the full-history one bit for bit and the plan honours its
  memory budget.
"""
import dataclasses
import sys

import numpy as np
import pytest

import fwi_inputs as fi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.linalg.norm(b))


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def _t(x, dev):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _acq(nz, nx, fs, nt, ns, two_rows=False, v_max=4000.0, dx=12.0, f_peak=25.0, nb=6):
    rec_iz = np.full(nx, 0 if fs else 1, np.int32)
    rec_ix = np.arange(nx, dtype=np.int32)
    if two_rows:  # a surface spread and a buried one
        rec_iz = np.concatenate([rec_iz, np.full(nx, nz // 2 + 1, np.int32)])
        rec_ix = np.concatenate([rec_ix, rec_ix])
    return fi.Acquisition(nz=nz, nx=nx, dz=10.0, dx=dx, dt=0.001, nt=nt, nb=nb, free_surface=fs, v_max=v_max,
                          src_iz=np.full(ns, 1, np.int32), src_ix=np.linspace(1, nx - 2, ns).astype(np.int32),
                          rec_iz=rec_iz, rec_ix=rec_ix, f_peak=f_peak, pml=True)


@pytest.mark.parametrize("nz,nx,fs,nt,two_rows,B,nb", [(9, 11, True, 160, False, 2, 6), (9, 11, False, 160, False, 1, 6),
                                                       (40, 50, True, 300, True, 2, 6), (37, 53, False, 300, True, 2, 6),
                                                       (62, 70, True, 400, False, 3, 6), (30, 36, False, 200, False, 2, 0),
                                                       (20, 24, False, 200, True, 2, 20), (16, 40, True, 200, False, 2, 20)])
def test_hbm_sweep_equals_lds_sweep(dev, nz, nx, fs, nt, two_rows, B, nb):
    """nb = 0: a PML geometry without layer cells (reflecting edges), whose layer-class tiles hold none.
    nb = 20: tiles lying mostly or wholly in the layer, whose waves list more layer cells than one pass of
    two per lane takes."""
    from paper_2603_16393_amd import FwiPlan

    acq = _acq(nz, nx, fs, nt, 3, two_rows, nb=nb)
    rng = np.random.default_rng(11 * nz + nx + B)
    w = _t(fi.ricker(nt, acq.dt, acq.f_peak), dev)
    lds = FwiPlan(acq, max_batch=B, device=dev, split=-1)
    hbm = FwiPlan(acq, max_batch=B, device=dev, force_path=1)
    ck = FwiPlan(acq, max_batch=B, device=dev, ckpt_every=37)
    infos = [dict(p.info) for p in (lds, hbm, ck)]
    _say(f"PML HBM sweep {nz}x{nx} fs={fs} B={B} nb={nb}: paths {[i['path'] for i in infos]}, "
         f"store modes {[i['store_mode'] for i in infos]}")
    assert [i["path"] for i in infos] == [2, 3, 3]
    assert infos[1]["store_mode"] == 0 and infos[2]["store_mode"] == 1 and infos[2]["ckpt_every"] == 37
    for call in range(3):
        v = _t(2000.0 + 1500.0 * rng.random((B, nz, nx)), dev)
        adj = _t(rng.standard_normal((B, acq.ns, acq.nr, nt)), dev)
        res = []
        for plan in (lds, hbm, ck):
            d = plan.forward(v, w, keep_for_adjoint=True)
            g = plan.adjoint_gradient(v, adj)
            torch.cuda.synchronize()
            assert plan.status() == 0
            res.append((d.clone(), g.clone()))
        for k in (1, 2):
            assert torch.equal(res[0][0], res[k][0]), f"traces differ (plan {k}, call {call})"
            assert torch.equal(res[0][1], res[k][1]), f"gradients differ (plan {k}, call {call})"
    for p in (lds, hbm, ck):
        p.close()


@pytest.mark.parametrize("ckpt", [0, 53])
def test_wide_field_vs_oracle(dev, ckpt):
    """120 x 160 (126 x 172 padded, 2 shots, 15 Hz, dx = dz = 10 m as in the 70 x 70 workload): too many cells
    for one workgroup, and a bottom layer of 1,032 cells is more than a row band's auxiliary update takes, so
    the plan sweeps it from HBM by itself.  (At 25 Hz with dx = 12 m these models drive the shifted synthetic
    traces so far below zero that the W2 adjoint source reaches 1e35, beyond FP32.)"""
    import oracle
    from paper_2603_16393_amd import FwiPlan

    nz, nx, nt = 120, 160, 500
    acq = _acq(nz, nx, True, nt, 2, v_max=4500.0, dx=10.0, f_peak=15.0)
    vt = fi.faulted_model(nz, nx, 3)
    v = np.stack([fi.faulted_model(nz, nx, s) for s in (0, 1)]).astype(np.float32)
    w = fi.ricker(nt, acq.dt, acq.f_peak).astype(np.float32)
    _say(f"PML HBM sweep 120x160 vs oracle, ckpt_every={ckpt}")
    dobs = oracle.forward(acq, _f32(vt[None]), _f32(w))[0].astype(np.float32)
    obs = oracle.w2_prepare(_f32(dobs), acq.dt)
    Jo, _, do, adjo = oracle.objective_and_gradient(acq, _f32(v), _f32(w), obs)
    adj_in = adjo.astype(np.float32)
    go = oracle.gradient(acq, _f32(v), _f32(w), _f32(adj_in))

    plan = FwiPlan(acq, max_batch=2, device=dev, ckpt_every=ckpt)
    info = dict(plan.info)
    plan.set_obs(_t(dobs, dev))
    vg = _t(v, dev)
    d = plan.forward(vg, _t(w, dev), keep_for_adjoint=True)
    J, _ = plan.w2_misfit(d, want_adjoint=False)
    g = plan.adjoint_gradient(vg, _t(adj_in, dev))
    torch.cuda.synchronize()
    assert plan.status() == 0
    d, J, g = d.cpu().numpy(), J.cpu().numpy(), g.cpu().numpy()
    plan.close()
    ed, eg = _rel(d, do), _rel(g, go)
    eJ = float(np.max(np.abs(J - Jo) / np.abs(Jo)))
    _say(f"  path {info['path']} store {info['store_mode']} ckpt {info['ckpt_every']}: traces {ed:.2e}, "
         f"J {eJ:.2e}, gradient {eg:.2e}")
    assert info["path"] == 3 and info["store_mode"] == (1 if ckpt else 0)
    assert ed <= 1e-4 and eJ <= 1e-5 and eg <= 1e-4


def _gradient(acq, v, vt, dev, **plan_kw):
    from paper_2603_16393_amd import FwiPlan

    w = _t(fi.ricker(acq.nt, acq.dt, acq.f_peak), dev)
    plan = FwiPlan(acq, max_batch=v.shape[0], device=dev, **plan_kw)
    dobs = plan.forward(_t(vt[None], dev), w, keep_for_adjoint=False)[0].contiguous()
    plan.set_obs(dobs)
    vg = _t(v, dev)
    d = plan.forward(vg, w, keep_for_adjoint=True)
    J, adj = plan.w2_misfit(d)
    g = plan.adjoint_gradient(vg, adj)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = dict(J=J.cpu().numpy(), g=g.cpu().numpy(), info=dict(plan.info))
    plan.close()
    return out


def test_full_size_checkpointed_equals_full_history(dev):
    nz, nx, nt = 400, 800, 4000
    acq = fi.surface_acquisition(nz, nx, ns=20, shot_cols=np.arange(20) * 40, nt=nt, nb=6, dt=8e-4, f_peak=10.0,
                                 v_max=5000.0)
    acq = dataclasses.replace(acq, pml=True).subset_shots([3, 17])
    vt = fi.large_lens_model(nz, nx, seed=1)
    v = fi.large_lens_model(nz, nx, seed=0)[None]
    budget = 4 << 30
    _say("PML full-size 400x800, 4000 steps, 2 shots: checkpointed under 4 GiB")
    a = _gradient(acq, v, vt, dev, mem_budget_bytes=budget, ckpt_every=100)
    assert a["info"]["path"] == 3 and a["info"]["store_mode"] == 1 and a["info"]["device_bytes"] <= budget
    _say("PML full-size: full history")
    b = _gradient(acq, v, vt, dev, force_path=1)
    assert b["info"]["path"] == 3 and b["info"]["store_mode"] == 0
    assert np.array_equal(a["J"], b["J"])
    assert np.array_equal(a["g"], b["g"])
    assert np.all(np.isfinite(a["g"])) and np.abs(a["g"]).max() > 0
