"""PML sweeps on the GPU vs the FP64 oracle (Sec. 2.1 absorbing boundary
realised by a PML; Sec. 6.1: 6 grid points on the left, right and bottom,
reflecting top).  Through the C ABI, on grids that use each per-thread slot
count of the sweep (2, 4 and 7 cells per thread), with and without the
reflecting top: forward traces (1e-4 relative L2), the W2 misfit of those
traces (1e-5), and the adjoint-state gradient for an adjoint source given to
both sides (1e-4): a random one on the small grids, the oracle's W2 adjoint
source on the 70 x 70 workload.  Observations come from the oracle.
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


def _t(x, dev):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _small_acq(nz, nx, fs, nt, ns, two_rows=False):
    rec_iz = np.full(nx, 0 if fs else 1, np.int32)
    rec_ix = np.arange(nx, dtype=np.int32)
    if two_rows:  # a surface spread and a buried one: several receivers share a thread of the sweep
        rec_iz = np.concatenate([rec_iz, np.full(nx, nz // 2 + 1, np.int32)])
        rec_ix = np.concatenate([rec_ix, rec_ix])
    return fi.Acquisition(nz=nz, nx=nx, dz=10.0, dx=12.0, dt=0.001, nt=nt, nb=6, free_surface=fs, v_max=4000.0,
                          src_iz=np.full(ns, 1, np.int32), src_ix=np.linspace(1, nx - 2, ns).astype(np.int32),
                          rec_iz=rec_iz, rec_ix=rec_ix, f_peak=25.0, pml=True)


@pytest.mark.parametrize("nz,nx,fs,nt,two_rows", [(9, 11, True, 160, False), (9, 11, False, 160, False),
                                                  (40, 50, True, 400, False), (37, 53, False, 300, False),
                                                  (62, 70, True, 500, False), (62, 70, True, 300, True),
                                                  (40, 50, False, 300, True)])
def test_pml_traces_and_gradient(dev, nz, nx, fs, nt, two_rows):
    import oracle
    from paper_2603_16393_amd import FwiPlan

    acq = _small_acq(nz, nx, fs, nt, 3, two_rows)
    rng = np.random.default_rng(nz * 1000 + nx + int(fs))
    v = (2000.0 + 1500.0 * rng.random((2, nz, nx))).astype(np.float32)
    w = fi.ricker(nt, acq.dt, acq.f_peak).astype(np.float32)
    adj = rng.standard_normal((2, acq.ns, acq.nr, nt)).astype(np.float32)
    do = oracle.forward(acq, _f32(v), _f32(w))
    go = oracle.gradient(acq, _f32(v), _f32(w), _f32(adj))

    plan = FwiPlan(acq, max_batch=2, device=dev)
    info = dict(plan.info)
    vg = _t(v, dev)
    d = plan.forward(vg, _t(w, dev), keep_for_adjoint=True)
    g = plan.adjoint_gradient(vg, _t(adj, dev))
    torch.cuda.synchronize()
    assert plan.status() == 0
    d, g = d.cpu().numpy(), g.cpu().numpy()
    plan.close()
    ed, eg = _rel(d, do), _rel(g, go)
    print(f"PML {nz}x{nx} fs={fs} nt={nt} receivers={acq.nr} padded {info['nzp']}x{info['nxp']} path={info['path']}: "
          f"traces {ed:.2e}, gradient {eg:.2e}", flush=True)
    assert info["path"] == 2
    assert ed <= 1e-4 and eg <= 1e-4


def test_pml_workload_70x70(dev):
    """The 70 x 70, 5-shot, 1000-sample workload with the paper's 6-cell PML."""
    import oracle
    from paper_2603_16393_amd import FwiPlan

    acq = dataclasses.replace(fi.operator_acquisition("Init").subset_shots([0, 2, 4, 6, 8]), nb=6, pml=True)
    vt = fi.faulted_model(70, 70, 1000)
    v = np.stack([fi.faulted_model(70, 70, s) for s in (0, 1)]).astype(np.float32)
    w = fi.ricker(acq.nt, acq.dt, acq.f_peak).astype(np.float32)
    dobs = oracle.forward(acq, _f32(vt[None]), _f32(w))[0].astype(np.float32)
    obs = oracle.w2_prepare(_f32(dobs), acq.dt)
    Jo, go, do, adjo = oracle.objective_and_gradient(acq, _f32(v), _f32(w), obs)
    adj_in = adjo.astype(np.float32)
    go = oracle.gradient(acq, _f32(v), _f32(w), _f32(adj_in))

    plan = FwiPlan(acq, max_batch=2, device=dev)
    plan.set_obs(_t(dobs, dev))
    vg = _t(v, dev)
    d = plan.forward(vg, _t(w, dev), keep_for_adjoint=True)
    J, _ = plan.w2_misfit(d, want_adjoint=False)
    g = plan.adjoint_gradient(vg, _t(adj_in, dev))
    torch.cuda.synchronize()
    assert plan.status() == 0
    info = dict(plan.info)
    d, J, g = d.cpu().numpy(), J.cpu().numpy(), g.cpu().numpy()
    plan.close()
    ed, eg = _rel(d, do), _rel(g, go)
    eJ = float(np.max(np.abs(J - Jo) / np.abs(Jo)))
    print(f"PML 70x70 nb=6: padded {info['nzp']}x{info['nxp']}: traces {ed:.2e}, J {eJ:.2e}, gradient {eg:.2e}",
          flush=True)
    sys.stdout.flush()
    assert info["path"] == 2 and (info["nzp"], info["nxp"]) == (76, 82)
    assert ed <= 1e-4 and eJ <= 1e-5 and eg <= 1e-4


@pytest.mark.parametrize("nz,nx,fs,nt,two_rows,B", [(70, 70, True, 1000, False, 16), (70, 70, True, 600, False, 1),
                                                    (70, 70, False, 400, False, 4), (40, 50, True, 300, True, 2),
                                                    (40, 50, False, 300, True, 2), (64, 48, True, 300, False, 3)])
def test_pml_row_bands_equal_whole_field(dev, nz, nx, fs, nt, two_rows, B):
    """The row-band sweep (several workgroups per field, halos exchanged every step) performs each cell's
    operations of the whole-field sweep and keeps its order of the D history: traces and gradients are
    equal bit for bit, on three calls in a row.  The buried spread of `two_rows` lies in the halo rows of
    a neighbouring band, so the adjoint's first values there are placed by that band itself."""
    from paper_2603_16393_amd import FwiPlan

    acq = _small_acq(nz, nx, fs, nt, 5 if B > 2 else 3, two_rows)
    rng = np.random.default_rng(7 * nz + nx + B)
    w = _t(fi.ricker(nt, acq.dt, acq.f_peak), dev)
    whole = FwiPlan(acq, max_batch=B, device=dev, split=-1)
    bands = FwiPlan(acq, max_batch=B, device=dev, split=1)
    iw, ib = dict(whole.info), dict(bands.info)
    print(f"PML {nz}x{nx} fs={fs} B={B}: bands {ib['lds_split']} (whole field {iw['lds_split']})", flush=True)
    assert iw["path"] == 2 and ib["path"] == 2 and iw["lds_split"] == 1 and ib["lds_split"] >= 2
    for call in range(3):
        v = _t(2000.0 + 1500.0 * rng.random((B, nz, nx)), dev)
        adj = _t(rng.standard_normal((B, acq.ns, acq.nr, nt)), dev)
        res = []
        for plan in (whole, bands):
            d = plan.forward(v, w, keep_for_adjoint=True)
            g = plan.adjoint_gradient(v, adj)
            torch.cuda.synchronize()
            assert plan.status() == 0
            res.append((d.clone(), g.clone()))
        assert torch.equal(res[0][0], res[1][0]), f"traces differ on call {call}"
        assert torch.equal(res[0][1], res[1][1]), f"gradients differ on call {call}"
    whole.close()
    bands.close()
