"""ctypes declarations of the C ABI in include/ns.h (argument marshalling only).

Every computation runs in libnsmi.so; this module never falls back to
Python arithmetic.  Importing it without a built library raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libnsmi.so")

NS_OK, NS_E_INVALID, NS_E_SHAPE, NS_E_HIP, NS_E_NOMEM, NS_E_NOT_SPD, NS_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "NS_OK", -1: "NS_E_INVALID", -2: "NS_E_SHAPE", -3: "NS_E_HIP", -4: "NS_E_NOMEM",
                -5: "NS_E_NOT_SPD", -6: "NS_E_UNSUPPORTED"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
KINDS = {"cmb_diag": 0, "cmb_block": 1, "shear": 2, "gauss": 3, "cmb_cv": 4}

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class NetDesc(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32),
        ("dims", c_int32_p),
        ("W", ctypes.POINTER(c_double_p)),
        ("b", ctypes.POINTER(c_double_p)),
        ("beta", ctypes.POINTER(c_double_p)),
        ("gamma", ctypes.POINTER(c_double_p)),
        ("in_shift", c_double_p),
        ("in_scale", c_double_p),
        ("out_mu", c_double_p),
        ("out_sigma", c_double_p),
    ]


class ModelDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("prior_kind", c_int32_p),
        ("prior_a", c_double_p),
        ("prior_b", c_double_p),
        ("n_nets", ctypes.c_int32),
        ("nets", ctypes.POINTER(NetDesc)),
        ("spec_log", c_int32_p),
        ("n_data", ctypes.c_int32),
        ("data", c_double_p),
        ("sigma", c_double_p),
        ("cov_blocks", c_double_p),
        ("sigma_pp", c_double_p),
        ("cov", c_double_p),
        ("n_bins", ctypes.c_int32),
        ("nz_mean", c_double_p),
        ("nz_sigma", ctypes.c_double),
        ("n_a", ctypes.c_int32),
        ("a_min", ctypes.c_double),
        ("n_z", ctypes.c_int32),
        ("k_min", ctypes.c_double),
        ("k_max", ctypes.c_double),
        ("n_k", ctypes.c_int32),
        ("ell_min", ctypes.c_double),
        ("ell_max", ctypes.c_double),
        ("n_ell", ctypes.c_int32),
        ("pidx", c_int32_p),
        ("pfix", c_double_p),
        ("mu", c_double_p),
        ("gsigma", c_double_p),
        ("z_interp", ctypes.c_int32),
    ]


class RunOpts(ctypes.Structure):
    _fields_ = [
        ("n_live", ctypes.c_int32),
        ("n_delete", ctypes.c_int32),
        ("n_inner", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("frac_remain", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("max_iter", ctypes.c_int32),
        ("n_replicates", ctypes.c_int32),
        ("checkpoint_path", ctypes.c_char_p),
        ("checkpoint_every", ctypes.c_int32),
        ("resume", ctypes.c_int32),
        ("speculate", ctypes.c_int32),
    ]


class RunResult(ctypes.Structure):
    _fields_ = [
        ("logz", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("sigma_skilling", ctypes.c_double),
        ("h", ctypes.c_double),
        ("n_iter", ctypes.c_int64),
        ("n_evals", ctypes.c_int64),
        ("n_stalls", ctypes.c_int64),
        ("n_dead", ctypes.c_int64),
        ("wall_s", ctypes.c_double),
        ("resumed_iter", ctypes.c_int64),
    ]


class HmcOpts(ctypes.Structure):
    _fields_ = [
        ("n_chains", ctypes.c_int32),
        ("n_iter", ctypes.c_int32),
        ("n_leapfrog", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("step", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class HmcResult(ctypes.Structure):
    _fields_ = [
        ("n_accept", ctypes.c_int64),
        ("n_left", ctypes.c_int64),
        ("n_grad", ctypes.c_int64),
        ("wall_s", ctypes.c_double),
    ]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("ns_model_create", ctypes.c_int, [ctypes.POINTER(ModelDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    ("ns_model_free", ctypes.c_int, [ctypes.c_void_p]),
    ("ns_model_dim", ctypes.c_int, [ctypes.c_void_p, c_int32_p]),
    ("ns_prior_transform", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_void_p]),
    ("ns_loglike_batch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    ("ns_theory_batch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]),
    ("ns_loglike_batch_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    ("ns_loglike_grad_batch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    ("ns_slice_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                     ctypes.c_void_p]),
    ("ns_run", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RunOpts), ctypes.POINTER(RunResult), ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("ns_hmc", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(HmcOpts), ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(HmcResult), ctypes.c_void_p]),
    ("ns_trace_enable", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("ns_trace_report", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    ("ns_tuning_report", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    ("ns_last_error", ctypes.c_char_p, []),
]

_lib = None


def lib():
    """The loaded libnsmi (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libnsmi.so not built at {LIB_PATH}; run python -m paper_2509_13307_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class NSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != NS_OK:
        raise NSError(code, lib().ns_last_error().decode())
