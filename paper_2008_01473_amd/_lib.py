"""ctypes declarations of the C ABI in include/lbm.h (argument marshalling only)."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

c_int, c_double, c_void_p, c_size_t, c_longlong = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, \
    ctypes.c_size_t, ctypes.c_longlong

LBM_OK, LBM_ERR_ARG, LBM_ERR_UNSUPPORTED, LBM_ERR_HIP, LBM_ERR_BLOWUP, LBM_ERR_DOMAIN, LBM_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6
LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_EOS_VDW, LBM_EOS_CS = 0, 1
LBM_STANDARD, LBM_IMPROVED = 0, 1
LBM_FORCE_CHEMPOT, LBM_FORCE_PTENSOR = 0, 1
LBM_FP64, LBM_FP32_DEV = 0, 1
LBM_BGK, LBM_MRT = 0, 1
LBM_STORES_STREAMING, LBM_STORES_DEVICE = 0, 1


class lbm_params(ctypes.Structure):
    _fields_ = [("lattice", c_int), ("nx", c_int), ("ny", c_int), ("nz", c_int),
                ("eos", c_int), ("a", c_double), ("b", c_double), ("R", c_double),
                ("T_over_Tc", c_double), ("kappa", c_double), ("tau", c_double),
                ("scheme", c_int), ("force_form", c_int), ("precision", c_int),
                ("rho_ref", c_double), ("pm_ref", c_double),
                ("collision", c_int), ("reserved", c_int),
                ("tau_e", c_double), ("tau_s", c_double), ("tau_q", c_double), ("nu", c_double),
                ("walls", c_int), ("reserved2", c_int), ("wall_u_bottom", c_double), ("wall_u_top", c_double),
                ("c0", c_double)]


class lbm_diag(ctypes.Structure):
    _fields_ = [("mass", c_double), ("mom", c_double * 3), ("max_u", c_double), ("mu_min", c_double),
                ("mu_max", c_double), ("step", c_longlong), ("status", c_int), ("reserved", c_int)]


P = ctypes.POINTER
# name -> (restype, argtypes); this list is the exported surface of include/lbm.h
SIGNATURES = {
    "lbm_create": (c_int, [P(lbm_params), c_void_p, P(c_void_p)]),
    "lbm_create_batch": (c_int, [P(lbm_params), c_int, c_void_p, P(c_void_p)]),
    "lbm_state_bytes": (c_size_t, [c_void_p]),
    "lbm_workspace_bytes": (c_size_t, [c_void_p]),
    "lbm_num_nodes": (c_longlong, [c_void_p]),
    "lbm_node_offset": (c_longlong, [c_void_p, c_int]),
    "lbm_count": (c_int, [c_void_p]),
    "lbm_bind": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "lbm_init": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lbm_step": (c_int, [c_void_p, c_int]),
    "lbm_prepare_steps": (c_int, [c_void_p, c_int]),
    "lbm_moments": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "lbm_diagnostics": (c_int, [c_void_p, P(lbm_diag)]),
    "lbm_get_f": (c_int, [c_void_p, c_void_p]),
    "lbm_set_f": (c_int, [c_void_p, c_void_p]),
    "lbm_get_state": (c_int, [c_void_p, c_void_p, P(c_longlong)]),
    "lbm_set_state": (c_int, [c_void_p, c_void_p, c_longlong]),
    "lbm_time": (c_longlong, [c_void_p]),
    "lbm_maxwell": (c_int, [c_int, c_double, c_double, c_double, c_double, P(c_double), P(c_double),
                            P(c_double), P(c_double)]),
    "lbm_critical_temperature": (c_double, [c_int, c_double, c_double, c_double]),
    "lbm_set_physics": (c_int, [c_void_p, c_int, c_double, c_double]),
    "lbm_adjoint_workspace_bytes": (c_size_t, [c_void_p]),
    "lbm_adjoint_segment": (c_int, [c_void_p, c_void_p, c_longlong, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p]),
    "lbm_adjoint_sweep": (c_int, [c_void_p, P(c_void_p), P(c_longlong), P(c_int), c_int, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "lbm_adjoint_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lbm_adjoint_step_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lbm_adjoint_noalloc_max_bytes": (c_size_t, []),
    "lbm_adjoint_fields": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lbm_adjoint_init": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lbm_set_tile_shape": (c_int, [c_void_p, c_int]),
    "lbm_get_tile_shape": (c_int, [c_void_p]),
    "lbm_num_tile_shapes": (c_int, [c_void_p]),
    "lbm_describe_tile_shape": (c_int, [c_void_p, c_int, P(c_int), P(c_int), P(c_int)]),
    "lbm_set_use_graphs": (c_int, [c_void_p, c_int]),
    "lbm_set_zchunk": (c_int, [c_void_p, c_int]),
    "lbm_get_zchunk": (c_int, [c_void_p]),
    "lbm_set_store_mode": (c_int, [c_void_p, c_int]),
    "lbm_get_store_mode": (c_int, [c_void_p]),
    "lbm_autotune": (c_int, [c_void_p, c_int, c_void_p]),
    "lbm_copy_kernel": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "lbm_error_string": (ctypes.c_char_p, [c_int]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_destroy": (None, [c_void_p]),
}

_LIB = None


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def lib():
    """Load liblbm.so (built in-tree by paper_2008_01473_amd.build); raises if absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2008_01473_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(code, what=""):
    if code < 0:
        L = lib()
        msg = L.lbm_last_error().decode() or L.lbm_error_string(code).decode()
        raise LBMError(code, f"{what}: {msg}" if what else msg)
    return code
