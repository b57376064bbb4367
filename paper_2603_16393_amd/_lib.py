"""ctypes binding of libfwi.so (the C ABI declared in include/fwi.h).

Argument marshalling only: every computation runs in the HIP kernels behind
the ABI.  Importing this module fails loudly when the library has not been
built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfwi.so")

c_int, c_double, c_size_t, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
c_int_p = ctypes.POINTER(ctypes.c_int)

FWI_OK, FWI_EINVAL, FWI_ECFL, FWI_ENOMEM, FWI_EHIP, FWI_ESTATE, FWI_EDEVICE = 0, -1, -2, -3, -4, -5, -6
FWI_W2_SCRATCH_PAIRS = 262144  # include/fwi.h

# Every symbol include/fwi.h declares.
EXPORTED = (
    "fwi_plan_create",
    "fwi_plan_create_ex",
    "fwi_plan_destroy",
    "fwi_plan_get_info",
    "fwi_set_obs",
    "fwi_forward",
    "fwi_w2_misfit",
    "fwi_w2_misfit_noalloc",
    "fwi_adjoint_gradient",
    "fwi_plan_history",
    "fwi_adjoint_gradient_of",
    "fwi_guidance_step",
    "fwi_l2_misfit",
    "fwi_tv_subgradient",
    "fwi_ddpm_step",
    "fwi_status",
    "fwi_plan_sweep_ms",
    "fwi_copy",
    "fwi_batch_create",
    "fwi_batch_destroy",
    "fwi_batch_get_info",
    "fwi_batch_sizes",
    "fwi_batch_forward",
    "fwi_batch_gradient",
    "fwi_batch_status",
    "fwi_error_string",
    "fwi_nn_gemm",
    "fwi_nn_mix_forward",
    "fwi_nn_mix_vjp",
    "fwi_nn_mlp_forward",
    "fwi_nn_mlp_vjp",
    "fwi_sur_shape",
    "fwi_sur_param_count",
    "fwi_sur_create",
    "fwi_sur_destroy",
    "fwi_sur_set_params",
    "fwi_sur_get_params",
    "fwi_sur_get_grads",
    "fwi_sur_get_adam",
    "fwi_sur_set_adam",
    "fwi_sur_set_fused_mlp",
    "fwi_sur_forward",
    "fwi_sur_backward",
    "fwi_sur_train_step",
    "fwi_judge",
    "fwi_mf_predict",
    "fwi_score_param_count",
    "fwi_score_create",
    "fwi_score_destroy",
    "fwi_score_set_params",
    "fwi_score_get_params",
    "fwi_score_get_grads",
    "fwi_score_get_adam",
    "fwi_score_set_adam",
    "fwi_score_forward",
    "fwi_score_backward",
    "fwi_score_train_step",
)


class Geometry(ctypes.Structure):
    _fields_ = [
        ("nz", c_int), ("nx", c_int), ("dz", c_double), ("dx", c_double), ("dt", c_double), ("nt", c_int),
        ("nb", c_int), ("free_surface", c_int), ("v_max", c_double), ("ns", c_int), ("src_iz", c_int_p),
        ("src_ix", c_int_p), ("nr", c_int), ("rec_iz", c_int_p), ("rec_ix", c_int_p), ("pml", c_int),
    ]


class W2Params(ctypes.Structure):
    _fields_ = [("k", c_double), ("eps_prime", c_double), ("n_xi", c_int), ("c_factor", c_double),
                ("squared", c_int), ("reduction", c_int)]


class L2Params(ctypes.Structure):
    _fields_ = [("sigma", c_double), ("k", c_double), ("normalize", c_int)]


class GuidanceParams(ctypes.Structure):
    _fields_ = [("rho0", c_double), ("c", c_double), ("tau", c_double), ("gamma", c_double), ("eps", c_double),
                ("kappa_max", c_double), ("unit_scale", c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nzp", c_int), ("nxp", c_int), ("path", c_int), ("store_mode", c_int), ("ckpt_every", c_int),
                ("max_batch", c_int), ("device_bytes", c_size_t), ("lds_tile_x", c_int), ("lds_tile_z", c_int),
                ("lds_split", c_int)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("force_path", c_int), ("ckpt_every", c_int), ("lds_tile_x", c_int), ("lds_tile_z", c_int),
                ("timing", c_int), ("split", c_int)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("autotune", c_int), ("gradients", c_int), ("bands", c_int)]


class BatchRequestInfo(ctypes.Structure):
    _fields_ = [("v_offset", c_size_t), ("wavelet_offset", c_size_t), ("trace_offset", c_size_t), ("nzp", c_int),
                ("nxp", c_int), ("kind", c_int), ("tile_x", c_int), ("tile_z", c_int), ("tuned", c_int),
                ("parts", c_int)]


class SurTrainParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("loss_k", ctypes.c_float), ("pair_weight", ctypes.c_float)]


class ScoreTrainParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class FwiError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = load().fwi_error_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what} failed: {msg} ({code})")
        self.code = code


_lib = None


def load():
    """Loads libfwi.so; raises if it is missing (build with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfwi.so not found at {LIB_PATH}; build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    L.fwi_plan_create.argtypes = [ctypes.POINTER(Geometry), c_int, c_size_t, ctypes.POINTER(P)]
    L.fwi_plan_create_ex.argtypes = [ctypes.POINTER(Geometry), c_int, c_size_t, ctypes.POINTER(PlanOptions),
                                     ctypes.POINTER(P)]
    L.fwi_plan_destroy.argtypes = [P]
    L.fwi_plan_get_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    L.fwi_set_obs.argtypes = [P, P, ctypes.POINTER(W2Params), P]
    L.fwi_forward.argtypes = [P, c_int, P, P, P, c_int, P]
    L.fwi_w2_misfit.argtypes = [P, c_int, P, P, P, P]
    L.fwi_w2_misfit_noalloc.argtypes = [P, c_int, P, P, P, P]
    L.fwi_adjoint_gradient.argtypes = [P, c_int, P, P, P, P, P]
    L.fwi_plan_history.argtypes = [P, ctypes.POINTER(ctypes.c_ulonglong)]
    L.fwi_adjoint_gradient_of.argtypes = [P, ctypes.c_ulonglong, c_int, P, P, P, P, P]
    L.fwi_l2_misfit.argtypes = [P, c_int, P, P, ctypes.POINTER(L2Params), P, P, P]
    L.fwi_tv_subgradient.argtypes = [c_int, c_int, c_int, P, P, c_double, P, P]
    L.fwi_ddpm_step.argtypes = [ctypes.c_long, P, P, P, c_double, c_double, c_double, c_double, P, P, P]
    L.fwi_guidance_step.argtypes = [c_int, c_int, c_int, P, P, P, P, ctypes.POINTER(GuidanceParams), P, P, P]
    L.fwi_status.argtypes = [P]
    L.fwi_plan_sweep_ms.argtypes = [P, P, P]
    L.fwi_copy.argtypes = [P, P, c_size_t, P]
    L.fwi_batch_create.argtypes = [c_int, P, ctypes.POINTER(BatchOptions), ctypes.POINTER(P)]
    L.fwi_batch_destroy.argtypes = [P]
    L.fwi_batch_get_info.argtypes = [P, c_int, ctypes.POINTER(BatchRequestInfo)]
    L.fwi_batch_sizes.argtypes = [P, ctypes.POINTER(c_size_t), ctypes.POINTER(c_size_t), ctypes.POINTER(c_size_t)]
    L.fwi_batch_forward.argtypes = [P, P, P, P, P]
    L.fwi_batch_gradient.argtypes = [P, P, P, P, P, P]
    L.fwi_batch_status.argtypes = [P]
    L.fwi_error_string.argtypes = [c_int]
    L.fwi_error_string.restype = ctypes.c_char_p
    cl, cf = ctypes.c_long, ctypes.c_float
    L.fwi_nn_gemm.argtypes = [c_int, c_int, c_int, c_int, P, cl, cl, c_int, P, cl, cl, c_int, P, P, cl, cl, cf, cf, P,
                              c_int, c_int, P, P]
    L.fwi_nn_mix_forward.argtypes = [cl, P, P, P, P]
    L.fwi_nn_mix_vjp.argtypes = [cl, P, P, P, P, P]
    L.fwi_nn_mlp_forward.argtypes = [cl, P, P, P, P, P, P, P, P]
    L.fwi_nn_mlp_vjp.argtypes = [cl, P, P, P, P, P, P, P]
    L.fwi_sur_set_fused_mlp.argtypes = [P, c_int]
    L.fwi_sur_shape.argtypes = [P]
    L.fwi_sur_param_count.argtypes = []
    L.fwi_sur_create.argtypes = [c_int, ctypes.POINTER(P)]
    L.fwi_sur_destroy.argtypes = [P]
    L.fwi_sur_set_params.argtypes = [P, P]
    L.fwi_sur_get_params.argtypes = [P, P]
    L.fwi_sur_get_grads.argtypes = [P, P]
    L.fwi_sur_get_adam.argtypes = [P, P, P, ctypes.POINTER(c_int)]
    L.fwi_sur_set_adam.argtypes = [P, P, P, c_int]
    L.fwi_sur_forward.argtypes = [P, c_int, P, P, P]
    L.fwi_sur_backward.argtypes = [P, c_int, P, P, c_int, P]
    L.fwi_sur_train_step.argtypes = [P, c_int, P, P, ctypes.POINTER(SurTrainParams), P, P]
    L.fwi_judge.argtypes = [c_int, c_int, P, P, P, P, P, P, P]
    L.fwi_mf_predict.argtypes = [c_int, c_int, P, P, P, P, P, P, P, P, P]
    L.fwi_score_param_count.argtypes = []
    L.fwi_score_create.argtypes = [c_int, ctypes.POINTER(P)]
    L.fwi_score_destroy.argtypes = [P]
    L.fwi_score_set_params.argtypes = [P, P]
    L.fwi_score_get_params.argtypes = [P, P]
    L.fwi_score_get_grads.argtypes = [P, P]
    L.fwi_score_get_adam.argtypes = [P, P, P, ctypes.POINTER(c_int)]
    L.fwi_score_set_adam.argtypes = [P, P, P, c_int]
    L.fwi_score_forward.argtypes = [P, c_int, P, P, P, P, P, P]
    L.fwi_score_backward.argtypes = [P, c_int, P, P, c_int, P]
    L.fwi_score_train_step.argtypes = [P, c_int, P, P, P, P, P, ctypes.POINTER(ScoreTrainParams), P, P]
    for name in EXPORTED:
        if name != "fwi_error_string":
            getattr(L, name).restype = c_int
    L.fwi_sur_param_count.restype = cl
    L.fwi_score_param_count.restype = cl
    _lib = L
    return _lib


def check(code: int, what: str):
    if code != FWI_OK:
        raise FwiError(code, what)
