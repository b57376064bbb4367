"""Runtime utilities of the C ABI on the GPU: the plain copy kernel and the
per-sweep event timing of a plan."""
import ctypes

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


@pytest.mark.parametrize("nbytes,off", [(0, 0), (1, 0), (15, 0), (16, 0), (1000003, 0), (4096, 3), (777, 5)])
def test_copy_is_exact(dev, nbytes, off):
    from paper_2603_16393_amd import _lib

    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device=dev)
    dst = torch.zeros_like(src)
    rc = _lib.load().fwi_copy(ctypes.c_void_p(dst.data_ptr() + off), ctypes.c_void_p(src.data_ptr() + off), nbytes,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(dst[off:off + nbytes], src[off:off + nbytes])
    assert int(dst[:off].sum()) == 0 and int(dst[off + nbytes:].sum()) == 0


def test_sweep_timing(dev):
    import fwi_inputs as fi
    from paper_2603_16393_amd import FwiPlan, _lib

    acq = fi.surface_acquisition(70, 70, ns=2, nt=400, nb=20)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    v = torch.tensor(np.stack([fi.faulted_model(70, 70, s) for s in range(3)]), dtype=torch.float32, device=dev)
    plain = FwiPlan(acq, max_batch=3, device=dev)
    with pytest.raises(_lib.FwiError) as e:
        plain.sweep_ms()
    assert e.value.code == _lib.FWI_ESTATE
    plan = FwiPlan(acq, max_batch=3, device=dev, timing=True)
    with pytest.raises(_lib.FwiError):
        plan.sweep_ms()  # nothing recorded yet
    d = plan.forward(v, w)
    plan.set_obs(d[0].contiguous())
    _, adj = plan.w2_misfit(d)
    plan.adjoint_gradient(v, adj)
    f0, a0 = plan.sweep_ms()
    assert f0 > 0 and a0 > 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        plan.forward(v, w, out=d)
    e1.record()
    torch.cuda.synchronize()
    f = ctypes.c_float()
    assert _lib.load().fwi_plan_sweep_ms(plan._h, ctypes.byref(f), None) == 0
    assert 0 < f.value <= e0.elapsed_time(e1) / 3 * 1.05 + 0.05
    # every count restarted: no adjoint since the first query, no forward since the second
    with pytest.raises(_lib.FwiError) as e:
        plan.sweep_ms()
    assert e.value.code == _lib.FWI_ESTATE
    plan.close()
    plain.close()


def test_adjoint_refuses_a_replaced_forward_history(dev):
    """Two misfit evaluations on one plan before one backward pass: the first one's history has been replaced,
    so its backward raises FWI_ESTATE instead of correlating with the second model's wavefields; in order
    (forward, backward, forward, backward) both gradients equal the plain calls'."""
    import fwi_inputs as fi
    from paper_2603_16393_amd import FwiPlan, FwiW2Loss, _lib

    acq = fi.surface_acquisition(40, 48, ns=2, nt=300, nb=12)
    w = torch.tensor(fi.ricker(acq.nt, acq.dt, acq.f_peak), dtype=torch.float32, device=dev)
    plan = FwiPlan(acq, max_batch=2, device=dev)
    vt = torch.tensor(fi.faulted_model(40, 48, 1000)[None], dtype=torch.float32, device=dev)
    plan.set_obs(plan.forward(vt, w, keep_for_adjoint=False)[0].contiguous())
    assert plan.history() == 0
    v1 = torch.tensor(np.stack([fi.faulted_model(40, 48, s) for s in (1, 2)]), dtype=torch.float32, device=dev)
    v2 = (v1 * 1.03).contiguous()
    a = v1.clone().requires_grad_(True)
    b = v2.clone().requires_grad_(True)
    J1 = FwiW2Loss.apply(a, plan, w)
    h1 = plan.history()
    J2 = FwiW2Loss.apply(b, plan, w)
    assert plan.history() == h1 + 1
    with pytest.raises(_lib.FwiError) as e:
        (J1.sum() + J2.sum()).backward()
    assert e.value.code == _lib.FWI_ESTATE
    # in order: each backward right after its forward
    ga = []
    for v in (v1, v2):
        x = v.clone().requires_grad_(True)
        FwiW2Loss.apply(x, plan, w).sum().backward()
        ga.append(x.grad.clone())
    for v, g in zip((v1, v2), ga):
        d = plan.forward(v, w)
        _, adj = plan.w2_misfit(d)
        assert torch.equal(plan.adjoint_gradient(v, adj), g)
    plan.forward(v1, w, keep_for_adjoint=False)
    assert plan.history() == 0
    torch.cuda.synchronize()
    plan.close()
