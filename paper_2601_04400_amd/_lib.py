"""ctypes loader for libshk.so (the HIP kernels behind include/shk.h).

There is no fallback: if the library is missing or was not built for this
machine the import of a solver fails loudly.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshk.so")

_d, _i, _p, _sz = ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t


class GridDesc(ctypes.Structure):
    """Mirror of shk_grid_desc."""
    _fields_ = [
        ("ndim", _i), ("nx", _i), ("ny", _i), ("nbatch", _i),
        ("x0", _d), ("x1", _d), ("y0", _d), ("y1", _d),
        ("prec", _i), ("gamma", _d), ("cfl", _d), ("weno_eps", _d),
        ("viscous", _i), ("mu", _d), ("prandtl", _d), ("nu_art", _d),
        ("bc", _i * 4), ("inflow_prim", _d * 4), ("ibm", _i), ("adjoint", _i), ("flux_net", _i),
        ("weno_char", _i),
    ]


# name -> (restype, argtypes)
_SIGS = {
    "shk_workspace_bytes": (_sz, [_p]),
    "shk_init_grid": (_i, [_p, _p, _sz, _p, _p]),
    "shk_destroy": (None, [_p]),
    "shk_set_stream": (_i, [_p, _p]),
    "shk_prim_to_cons": (_i, [_p, _p, _p]),
    "shk_prim_to_cons_vjp": (_i, [_p, _p, _p, _p, _p]),
    "shk_set_ib_levelset": (_i, [_p, _p, _i]),
    "shk_ib_ghost_count": (_i, [_p, _p]),
    "shk_ib_classes": (_i, [_p, _p]),
    "shk_rhs": (_i, [_p, _p, _p]),
    "shk_ib_fill": (_i, [_p, _p]),
    "shk_rk3_step": (_i, [_p, _p, _p, _p]),
    "shk_rhs_adjoint": (_i, [_p, _p, _p, _p, _p]),
    "shk_rk3_step_adjoint": (_i, [_p, _p, _p, _p, _p]),
    "shk_rk3_step_record": (_i, [_p, _p, _p, _p, _p]),
    "shk_rk3_step_adjoint_tape": (_i, [_p, _p, _p, _p, _p]),
    "shk_rk3_steps_record": (_i, [_p, _p, _i, _p, _p]),
    "shk_set_params": (_i, [_p, _d, _p]),
    "shk_rk3_steps_adjoint_tape": (_i, [_p, _p, _i, _p, _p, _p]),
    "shk_set_flux_net": (_i, [_p, _p, _p, _p, ctypes.c_float, _i]),
    "shk_set_flux_net_grad": (_i, [_p, _p]),
    "shk_flux_net_eval": (_i, [_p, _p, _p]),
    "shk_flux_net_vjp": (_i, [_p, _p, _p, _p, _p]),
    "shk_flux_net_pack": (_i, [_p, _p, _p, _p]),
    "shk_set_flux_cnn": (_i, [_p, _p, _p, _p, ctypes.c_float, _i]),
    "shk_flux_cnn_eval": (_i, [_p, _p, _p]),
    "shk_flux_cnn_vjp": (_i, [_p, _p, _p, _p, _p]),
    "shk_flux_cnn_images": (_i, [_p, _p, _p, _p]),
    "shk_flux_cnn_pack": (_i, [_p, _p, _p, _p]),
    "shk_adam": (_i, [_p, _p, _p, _p, _i, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _i, _p]),
    "shk_restrict": (_i, [_p, _p, _i, _i, _i, _i, _i, _p]),
    "shk_mse": (_i, [_p, _p, _p, _d, ctypes.c_longlong, _i, _p, _p, _p]),
    "shk_mse_noalloc": (_i, [_p, _p, _p, _d, ctypes.c_longlong, _i, _p, _p]),
    "shk_set_time": (_i, [_p, _d, _d]),
    "shk_get_time": (_i, [_p, _i, _p, _p, _p]),
    "shk_poll_faults": (_i, [_p, _p, _p]),
    "shk_profile": (_i, [_p, _i]),
    "shk_profile_read": (_i, [_p, _p, _p]),
    "shk_last_error": (ctypes.c_char_p, [_p]),
    "shk_status_string": (ctypes.c_char_p, [_i]),
    "shk_normal_shock_state": (_i, [_d, _d, _d, _d, _p, _p, _p]),
}

# Every symbol declared in include/shk.h (checked by the ABI test).
EXPORTS = tuple(_SIGS)

_lib = None


def lib():
    """Load libshk.so once; raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2601_04400_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class ShkError(RuntimeError):
    pass


def check(status, handle=None, what=""):
    if status != 0:
        name = lib().shk_status_string(status).decode()
        msg = lib().shk_last_error(handle).decode() if handle else ""
        raise ShkError(f"{what}: {name} {msg}".strip())
