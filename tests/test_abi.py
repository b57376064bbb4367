"""The C ABI library loads and exports every symbol include/fwi.h declares
(no GPU needed); host-side argument validation returns before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fwi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|long|const char\*)\s+(fwi_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("fwi_forward", "fwi_w2_misfit", "fwi_adjoint_gradient", "fwi_guidance_step", "fwi_set_obs",
              "fwi_plan_create", "fwi_plan_destroy", "fwi_status"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    names = _declared()
    assert set(names) == set(_lib.EXPORTED)
    for n in names:
        assert hasattr(L, n), n
    assert L.fwi_error_string(-2).decode().startswith("CFL")


def _geom(nz=10, nx=10, dt=1e-3, vmax=4500.0, src=(0, 5), recs=((0, 1), (0, 2))):
    from paper_2603_16393_amd import _lib

    keep = [np.array([src[0]], np.int32), np.array([src[1]], np.int32),
            np.array([r[0] for r in recs], np.int32), np.array([r[1] for r in recs], np.int32)]
    p = [k.ctypes.data_as(_lib.c_int_p) for k in keep]
    g = _lib.Geometry(nz, nx, 10.0, 10.0, dt, 100, 4, 1, vmax, 1, p[0], p[1], len(recs), p[2], p[3])
    return g, keep


@pytest.mark.parametrize("kw,code", [
    (dict(dt=2e-3), -2),                 # CFL: 4500 * 2e-3 / 10 = 0.9 > 0.5546
    (dict(src=(10, 5)), -1),             # source outside the model
    (dict(recs=((0, 1), (0, 1))), -1),   # duplicate receiver node
    (dict(recs=((0, 1), (3, 10))), -1),  # receiver outside
    (dict(vmax=-1.0), -1),
])
def test_plan_create_validation(kw, code):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    g, keep = _geom(**kw)
    h = ctypes.c_void_p()
    assert L.fwi_plan_create(ctypes.byref(g), 1, 0, ctypes.byref(h)) == code
    assert not h.value


def test_guidance_validation():
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    bad = _lib.GuidanceParams(1.0, 0.0, 0.0, 0.5, 1e-4, 0.0, 1.0)  # c = 0
    x = ctypes.c_void_p(16)
    assert L.fwi_guidance_step(1, 4, 4, x, x, x, x, ctypes.byref(bad), x, None, None) == -1
    ok = _lib.GuidanceParams(1.0, 0.1, 0.0, 0.5, 1e-4, 0.0, 1.0)
    assert L.fwi_guidance_step(0, 4, 4, None, None, None, None, ctypes.byref(ok), None, None, None) == 0


def test_mlp_and_surrogate_option_validation():
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    x = ctypes.c_void_p(256)
    assert L.fwi_nn_mlp_forward(-1, x, x, x, x, x, x, x, None) == -1
    assert L.fwi_nn_mlp_forward(0, None, None, None, None, None, None, None, None) == 0
    assert L.fwi_nn_mlp_forward(16, x, x, None, x, x, x, x, None) == -1
    assert L.fwi_nn_mlp_forward(16, ctypes.c_void_p(258), x, x, x, x, x, x, None) == -1  # not 16-byte aligned
    assert L.fwi_nn_mlp_vjp(-5, x, x, x, x, x, x, None) == -1
    assert L.fwi_nn_mlp_vjp(0, None, None, None, None, None, None, None) == 0
    assert L.fwi_nn_mlp_vjp(16, x, x, x, x, x, None, None) == -1
    assert L.fwi_sur_set_fused_mlp(None, 1) == -1
    assert L.fwi_nn_mix_forward(-1, x, x, x, None) == -1
    assert L.fwi_nn_mix_forward(0, None, None, None, None) == 0
    assert L.fwi_nn_mix_forward(2, x, ctypes.c_void_p(258), x, None) == -1       # not 16-byte aligned
    assert L.fwi_nn_mix_vjp(2, x, x, None, x, None) == -1


def test_variant_entry_point_validation():
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    x = ctypes.c_void_p(256)
    lp = _lib.L2Params(0.05, 0.0, 0)
    assert L.fwi_l2_misfit(None, 1, x, x, ctypes.byref(lp), x, x, None) == -1
    assert L.fwi_tv_subgradient(-1, 4, 4, x, None, 1.0, ctypes.c_void_p(512), None) == -1
    assert L.fwi_tv_subgradient(1, 4, 0, x, None, 1.0, ctypes.c_void_p(512), None) == -1
    assert L.fwi_tv_subgradient(1, 4, 4, x, None, 1.0, x, None) == -1          # out aliases v
    assert L.fwi_tv_subgradient(1, 4, 4, x, None, float("inf"), ctypes.c_void_p(512), None) == -1
    assert L.fwi_tv_subgradient(0, 4, 4, None, None, 1.0, None, None) == 0


def test_product_has_no_oracle_or_cpu_path():
    """The product package never imports the oracle, and the HIP library is required."""
    pkg = os.path.join(ROOT, "paper_2603_16393_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "fwi_oracle" not in src, f


def _pml_geom(nz, nx, recs, pml=1, nb=6):
    from paper_2603_16393_amd import _lib

    keep = [np.array([0], np.int32), np.array([nx // 2], np.int32),
            np.array([r[0] for r in recs], np.int32), np.array([r[1] for r in recs], np.int32)]
    p = [k.ctypes.data_as(_lib.c_int_p) for k in keep]
    g = _lib.Geometry(nz, nx, 10.0, 10.0, 1e-3, 100, nb, 1, 4500.0, 1, p[0], p[1], len(recs), p[2], p[3], pml)
    return g, keep


@pytest.mark.parametrize("case", ["flag", "lds_checkpoint", "lds_tile", "split", "split_hbm", "batch"])
def test_pml_plan_validation(case):
    """The PML layer (Sec. 6.1) runs on its LDS-resident sweeps or on its HBM
    sweep: every request neither can serve is refused on the host with
    FWI_EINVAL."""
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    h = ctypes.c_void_p()
    recs = tuple((0, i) for i in range(8))
    if case == "flag":
        g, keep = _pml_geom(20, 20, recs, pml=2)
        assert L.fwi_plan_create(ctypes.byref(g), 1, 0, ctypes.byref(h)) == -1
    elif case == "batch":
        g, keep = _pml_geom(20, 20, recs)
        geoms = (_lib.Geometry * 1)(g)
        assert L.fwi_batch_create(1, geoms, None, ctypes.byref(h)) == -1
    else:
        g, keep = _pml_geom(20, 20, recs)
        opts = {"lds_checkpoint": (0, 10, 0, 0, 0, 0),  # the LDS-resident PML sweeps keep the full history
                "lds_tile": (-1, 0, 3, 3, 0, 0),        # register tiles belong to the sponge's LDS sweep
                "split": (-1, 0, 0, 0, 0, 1),           # 26 padded rows: too few for two row bands
                "split_hbm": (1, 0, 0, 0, 0, 1)}[case]  # the HBM sweep has no row bands
        o = _lib.PlanOptions(*opts)
        assert L.fwi_plan_create_ex(ctypes.byref(g), 1, 0, ctypes.byref(o), ctypes.byref(h)) == -1
    assert not h.value


@pytest.mark.parametrize("case", ["tiled", "checkpoint", "too_big"])
def test_pml_hbm_requests_pass_host_validation(case):
    """Requests the LDS-resident PML sweeps cannot serve go to the HBM sweep:
    the host accepts them (without a GPU the plan then fails on device
    memory, not on validation)."""
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    h = ctypes.c_void_p()
    recs = tuple((0, i) for i in range(8))
    if case == "too_big":
        g, keep = _pml_geom(120, 120, recs)  # 126 x 132 padded cells: more than one workgroup's LDS
        rc = L.fwi_plan_create(ctypes.byref(g), 1, 0, ctypes.byref(h))
    else:
        g, keep = _pml_geom(20, 20, recs)
        o = _lib.PlanOptions(1 if case == "tiled" else -1, 10 if case == "checkpoint" else 0, 0, 0, 0, 0)
        rc = L.fwi_plan_create_ex(ctypes.byref(g), 1, 0, ctypes.byref(o), ctypes.byref(h))
    assert rc != _lib.FWI_EINVAL
    if rc == 0:
        info = _lib.PlanInfo()
        assert L.fwi_plan_get_info(h, ctypes.byref(info)) == 0
        assert info.path in (2, 3)
        assert L.fwi_plan_destroy(h) == 0


@pytest.mark.parametrize("beta,abar,abar_prev,sigma", [(0.0, 0.5, 0.6, 0.0), (0.1, 0.7, 0.6, 0.0),
                                                      (0.1, 0.5, 1.5, 0.0), (0.1, 0.5, 0.6, -1.0)])
def test_ddpm_step_validation(beta, abar, abar_prev, sigma):
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    x = ctypes.c_void_p(256)
    assert L.fwi_ddpm_step(8, x, None, None, beta, abar, abar_prev, sigma, x, x, None) == -1
    ok = L.fwi_ddpm_step(0, None, None, None, 0.1, 0.5, 0.6, 0.0, None, None, None)
    assert ok == 0


def test_history_entry_points_validate_on_the_host():
    from paper_2603_16393_amd import _lib

    L = _lib.load()
    h = ctypes.c_ulonglong(7)
    assert L.fwi_plan_history(None, ctypes.byref(h)) == _lib.FWI_EINVAL
    assert L.fwi_adjoint_gradient_of(None, 1, 1, None, None, None, None, None) == _lib.FWI_EINVAL


def test_noalloc_capacity_matches_the_header():
    from paper_2603_16393_amd import _lib

    txt = open(os.path.join(ROOT, "include", "fwi.h")).read()
    m = re.search(r"#define FWI_W2_SCRATCH_PAIRS (\d+)", txt)
    assert m and int(m.group(1)) == _lib.FWI_W2_SCRATCH_PAIRS
    L = _lib.load()
    assert L.fwi_w2_misfit_noalloc(None, 1, None, None, None, None) == _lib.FWI_EINVAL
