"""The allocation-free misfit entry point (fwi_w2_misfit_noalloc) through the
C ABI: the same J and adjoint source as fwi_w2_misfit, bit for bit, on two
calls in a row (the second with a smaller batch on another plan), and a clear
error for a batch beyond its fixed scratch."""
import ctypes

import numpy as np
import pytest

import fwi_inputs as fi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    return d


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pair(plan, d, dev):
    """(J, adj) from fwi_w2_misfit and from fwi_w2_misfit_noalloc on the same traces."""
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    B = d.shape[0]
    out = []
    for fn in (L.fwi_w2_misfit, L.fwi_w2_misfit_noalloc):
        J = torch.full((B,), float("nan"), dtype=torch.float64, device=dev)
        adj = torch.full_like(d, float("nan"))
        rc = fn(plan._h, B, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                ctypes.c_void_p(adj.data_ptr()), _stream())
        assert rc == _lib.FWI_OK, rc
        out.append((J, adj))
    torch.cuda.synchronize()
    return out


def _setup(dev, nz, nx, ns, nt, B, seed):
    from paper_2603_16393_amd import FwiPlan

    acq = fi.surface_acquisition(nz, nx, ns=ns, nt=nt, nb=10)
    plan = FwiPlan(acq, max_batch=B, device=dev)
    w = torch.tensor(fi.ricker(nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    vt = torch.tensor(fi.faulted_model(nz, nx, seed)[None], dtype=torch.float32, device=dev)
    plan.set_obs(plan.forward(vt, w, keep_for_adjoint=False)[0].contiguous())
    v = torch.tensor(np.stack([fi.faulted_model(nz, nx, seed + 1 + b) for b in range(B)]), dtype=torch.float32,
                     device=dev)
    d = plan.forward(v, w, keep_for_adjoint=False)
    return plan, d


def test_noalloc_misfit_equals_the_plan_workspace_misfit(dev):
    print("noalloc: call 1 (B=6, 4 shots x 48 receivers, nt=600)", flush=True)
    plan, d = _setup(dev, 40, 48, 4, 600, 6, 11)
    (J0, a0), (J1, a1) = _pair(plan, d, dev)
    assert torch.isfinite(J1).all() and torch.isfinite(a1).all()
    assert torch.equal(J0, J1) and torch.equal(a0, a1)
    plan.close()
    print("noalloc: call 2 (B=2, 3 shots x 31 receivers, nt=450)", flush=True)
    plan2, d2 = _setup(dev, 26, 31, 3, 450, 3, 23)
    d2 = d2[:2].contiguous()
    (J0, a0), (J1, a1) = _pair(plan2, d2, dev)
    assert torch.isfinite(J1).all() and torch.isfinite(a1).all()
    assert torch.equal(J0, J1) and torch.equal(a0, a1)
    plan2.close()


def test_noalloc_rejects_a_batch_beyond_its_scratch(dev):
    from paper_2603_16393_amd import FwiPlan, _lib

    nx, ns = 700, 20
    B = _lib.FWI_W2_SCRATCH_PAIRS // (ns * nx) + 1  # B * ns * nr just above the capacity
    acq = fi.surface_acquisition(6, nx, ns=ns, nt=4, nb=2)
    plan = FwiPlan(acq, max_batch=B, device=dev)
    d = torch.zeros(1, dtype=torch.float32, device=dev)
    J = torch.zeros(1, dtype=torch.float64, device=dev)
    rc = _lib.load().fwi_w2_misfit_noalloc(plan._h, B, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                                           None, _stream())
    assert rc == _lib.FWI_ENOMEM
    plan.close()
