"""ctypes declarations of the C ABI in include/best.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbest.so")

BEST_OK, BEST_EINVAL, BEST_ENOMEM, BEST_EHIP, BEST_ENOTPD, BEST_ESTATE = range(6)
BEST_FP64, BEST_FP32, BEST_FP16, BEST_BF16 = range(4)
BEST_MH, BEST_MALA, BEST_HMC, BEST_AIES, BEST_NUTS, BEST_DE = range(6)
BEST_NUTS_MAX_DEPTH = 12
BEST_INIT_UNIFORM, BEST_INIT_REPLICATED, BEST_INIT_GAUSSIAN, BEST_INIT_HYPERSPHERE = range(4)
BEST_HOST_PTRS = 1
BEST_AOS = 2
BEST_ESS_OK, BEST_ESS_UNTRUNCATED, BEST_ESS_FROZEN = range(3)

PRECISIONS = {"fp64": BEST_FP64, "fp32": BEST_FP32, "fp16": BEST_FP16, "bf16": BEST_BF16}
SAMPLERS = {"mh": BEST_MH, "mala": BEST_MALA, "hmc": BEST_HMC, "aies": BEST_AIES,
            "nuts": BEST_NUTS, "de": BEST_DE}

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


class PlainModel(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("n_terms", C.c_int32),
                ("xgrid", _dp), ("data", _dp), ("inv_sigma2", _dp),
                ("a", _dp), ("g", _dp), ("p", _dp), ("k", _dp), ("gamma0", _dp),
                ("center", _dp), ("invscale", _dp)]


class Problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("lower", _dp), ("upper", _dp),
                ("gauss_coef", C.c_double), ("gauss_mean", _dp), ("gauss_prec", _dp),
                ("twist_u", C.c_int32), ("twist_v", C.c_int32),
                ("twist_beta", C.c_double), ("twist_center", C.c_double),
                ("twist_kappa", C.c_double),
                ("width", C.c_int32), ("n_hidden", C.c_int32), ("mlp_params", _dp),
                ("in_center", _dp), ("in_invscale", _dp),
                ("mlp_coef", C.c_double), ("offset", C.c_double),
                ("plain_mode", C.c_int32), ("train_lo", _dp), ("train_hi", _dp),
                ("plain", C.POINTER(PlainModel)),
                ("box_penalty", C.c_int32), ("penalty_width", C.c_double)]


class Config(C.Structure):
    _fields_ = [("n_chains", C.c_int64), ("precision", C.c_int32), ("seed", C.c_uint64),
                ("init", C.c_int32), ("init_point", _dp), ("init_scale", C.c_double),
                ("stream", C.c_void_p), ("chains_per_block", C.c_int32)]


class StepParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("mh_scale", C.c_double), ("stretch_a", C.c_double),
                ("n_leapfrog", C.c_int32), ("thin", C.c_int32), ("record", _fp),
                ("record_capacity", C.c_int64), ("adapt_eps", C.c_int32),
                ("target_accept", C.c_double), ("max_depth", C.c_int32),
                ("de_sigma", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("accepted", C.c_int64), ("evals", C.c_int64), ("n_nonfinite", C.c_int64),
                ("n_oob", C.c_int64), ("n_recorded", C.c_int64),
                ("sum_accept_prob", C.c_double), ("ms", C.c_double), ("eps", C.c_double),
                ("eps_bar", C.c_double)]


class AdaptParams(C.Structure):
    _fields_ = [("samples", _fp), ("n_samples", C.c_int64), ("update_mean", C.c_int32),
                ("reset_da", C.c_int32), ("finalize_da", C.c_int32),
                ("target_accept", C.c_double)]


class AdaptInfo(C.Structure):
    _fields_ = [("jitter", C.c_double), ("logdet", C.c_double), ("eps", C.c_double)]


EXPORTS = {
    "best_init": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Problem), C.POINTER(Config)]),
    "best_destroy": (None, [C.c_void_p]),
    "best_strerror": (C.c_char_p, [C.c_int]),
    "best_last_error": (C.c_char_p, [C.c_void_p]),
    "best_mlp_nparams": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32]),
    "best_logL_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                 C.c_uint32]),
    "best_logL_param_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_void_p]),
    "best_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(StepParams),
                            C.POINTER(StepStats)]),
    "best_adapt": (C.c_int, [C.c_void_p, C.POINTER(AdaptParams), C.POINTER(AdaptInfo)]),
    "best_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32]),
    "best_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32]),
    "best_get_whitening": (C.c_int, [C.c_void_p, _dp, _dp]),
    "best_set_whitening": (C.c_int, [C.c_void_p, _dp, _dp]),
    "best_get_step_counter": (C.c_uint64, [C.c_void_p]),
    "best_set_step_counter": (C.c_int, [C.c_void_p, C.c_uint64]),
    "best_set_step_size": (C.c_int, [C.c_void_p, C.c_double]),
    "best_set_step_multipliers": (C.c_int, [C.c_void_p, _dp]),
    "best_reinit": (C.c_int, [C.c_void_p, C.c_int32, _dp, C.c_double]),
    "best_set_mlp": (C.c_int, [C.c_void_p, _dp, C.c_double, C.c_double]),
    "best_ess": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, _dp, C.c_void_p]),
    "best_ess_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, _dp, C.c_void_p]),
    "best_rhat": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, _dp]),
    "best_credible": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_double, _dp,
                                _dp, _dp, _dp, _dp, _dp, _dp]),
    "best_sliced_wasserstein": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                          C.c_void_p, C.c_int64, C.c_int64, C.c_int32,
                                          C.c_uint64, _dp, _dp, _dp]),
    "best_trainer_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32,
                                      _dp, C.c_int32, C.c_void_p]),
    "best_trainer_destroy": (None, [C.c_void_p]),
    "best_train_epoch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                   C.c_int32, C.c_double, C.c_double, C.c_int64, C.c_int64,
                                   _dp]),
    "best_train_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, _dp, _dp]),
    "best_trainer_get_params": (C.c_int, [C.c_void_p, _dp]),
    "best_trainer_last_error": (C.c_char_p, [C.c_void_p]),
    "best_standardise": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, _dp, C.c_void_p]),
    "best_normalise_inputs": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, _dp, _dp, C.c_void_p,
                                        C.c_void_p]),
    "best_importance_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, _dp,
                                          C.c_void_p]),
}

_LIB = None


def load(path: str | None = None):
    """Load libbest.so (built in-tree by paper_2606_04895_amd.build); raises if missing."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    try:  # load torch's HIP runtime first so the process holds a single runtime
        import torch  # noqa: F401
    except Exception:  # pragma: no cover - torch absent
        pass
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing "
                           "(run python -m paper_2606_04895_amd.build)")
    lib = C.CDLL(p)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib
