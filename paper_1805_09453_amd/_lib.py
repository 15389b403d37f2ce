"""ctypes declarations for libgprox.so (include/gprox.h).  Marshalling only."""
import ctypes
import os

from .build import LIB

c_int, c_double, c_void_p, c_longlong = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_longlong

GP_OK, GP_ENOTCONV, GP_EINVAL, GP_EMASS, GP_ENOMEM, GP_EHIP, GP_EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5
GP_KIND_ROF, GP_KIND_EMD = 0, 1
GP_NORM_ISO, GP_NORM_ANISO = 0, 1


class gp_opts(ctypes.Structure):
    _fields_ = [("tau", c_double), ("sigma", c_double), ("tol", c_double), ("max_iter", c_int),
                ("check_every", c_int), ("norm", c_int), ("warm_start", c_int), ("ergodic", c_int)]


class gp_report(ctypes.Structure):
    _fields_ = [("iters", c_int), ("converged", c_int), ("primal", c_double), ("dual", c_double),
                ("rel_gap", c_double), ("div_residual", c_double), ("seconds_setup", c_double),
                ("seconds_loop", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gp_state(ctypes.Structure):
    _fields_ = [("kind", c_int), ("ny", c_int), ("nx", c_int), ("norm", c_int), ("h", c_double),
                ("lam", c_double), ("tau", c_double), ("sigma", c_double), ("f", c_void_p),
                ("gpsi", c_void_p), ("u", c_void_p), ("p", c_void_p), ("pbar", c_void_p),
                ("iter", c_longlong)]


class gp_instance(ctypes.Structure):
    _fields_ = [("kind", c_int), ("ny", c_int), ("nx", c_int), ("h", c_double), ("lam", c_double),
                ("tau", c_double), ("in0", c_void_p), ("in1", c_void_p), ("out", c_void_p), ("phi", c_void_p)]


class gp_rof_rule(ctypes.Structure):
    _fields_ = [("tv", c_double), ("grad_l2", c_double), ("tv_bound", c_double), ("tau", c_double),
                ("tau_continuum", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ws_report(ctypes.Structure):
    _fields_ = [("used_warm", c_int), ("fallback", c_int), ("warm_iters", c_int), ("d0", c_double),
                ("seconds_predict", c_double), ("seconds_total", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gp_kstat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("calls", c_longlong), ("dropped", c_longlong),
                ("total_ms", c_double), ("bytes", c_double)]


_SIGS = {
    "gp_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_void_p]),
    "gp_destroy": (c_int, [c_void_p]),
    "gp_strerror": (ctypes.c_char_p, [c_int]),
    "gp_last_error": (ctypes.c_char_p, [c_void_p]),
    "dct_poisson": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_double, c_double]),
    "dct_poisson_f64": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_double, c_double]),
    "dct_poisson_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_int, c_double, c_double, c_void_p]),
    "rof_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_double, c_double,
                          ctypes.POINTER(gp_opts), ctypes.POINTER(gp_report)]),
    "emd_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_double,
                          ctypes.POINTER(gp_opts), ctypes.POINTER(gp_report)]),
    "dct_poisson3": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_double, c_double]),
    "dct_poisson3_f64": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_double, c_double]),
    "rof3_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_double, c_double,
                           ctypes.POINTER(gp_opts), ctypes.POINTER(gp_report)]),
    "emd3_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_double,
                           ctypes.POINTER(gp_opts), ctypes.POINTER(gp_report)]),
    "emd_setup": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_double]),
    "rof_step_rule": (c_int, [c_void_p, c_void_p, c_int, c_int, c_double, c_double, c_double, c_int,
                              ctypes.POINTER(gp_rof_rule)]),
    "emd_step_rule_singular": (c_double, [c_double, c_double]),
    "pd_step": (c_int, [c_void_p, ctypes.POINTER(gp_state), c_int]),
    "pd_gap": (c_int, [c_void_p, ctypes.POINTER(gp_state), ctypes.POINTER(gp_report)]),
    "gp_batch_solve": (c_int, [c_void_p, ctypes.POINTER(gp_instance), c_int, ctypes.POINTER(gp_opts),
                               ctypes.POINTER(gp_report)]),
    "gp_get_shape": (c_int, [c_void_p, c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                             ctypes.POINTER(c_int)]),
    "gp_set_shape": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "gp_get_radix_plan": (c_int, [c_void_p, c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "gp_set_radix_plan": (c_int, [c_void_p, c_int, c_int, ctypes.POINTER(c_int), c_int]),
    "ws_param_count": (c_longlong, []),
    "ws_create": (c_int, [c_void_p, ctypes.POINTER(c_void_p), c_int, c_int, c_int]),
    "ws_destroy": (c_int, [c_void_p]),
    "ws_set_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ws_get_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ws_predict": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "ws_grads": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double, c_void_p,
                         ctypes.POINTER(c_double)]),
    "ws_adam": (c_int, [c_void_p, c_void_p, c_double]),
    "ws_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double, c_double, c_void_p]),
    "ws_load_params": (c_int, [c_void_p, c_void_p, ctypes.c_char_p]),
    "ws_save_params": (c_int, [c_void_p, c_void_p, ctypes.c_char_p]),
    "ws_downsample": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "ws_upsample": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
    "ws_emd_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_double,
                             ctypes.POINTER(gp_opts), ctypes.POINTER(gp_report), ctypes.POINTER(ws_report)]),
    "gp_profile": (c_int, [c_void_p, c_int]),
    "gp_profile_read": (c_int, [c_void_p, ctypes.POINTER(gp_kstat), c_int, ctypes.POINTER(c_int)]),
}

_lib = None


def load():
    """Load the in-tree libgprox.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"libgprox.so not found at {LIB}: run paper_1805_09453_amd.build.build() first")
        lib = ctypes.CDLL(LIB)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
