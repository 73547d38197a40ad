"""ctypes binding of libdope.so (include/dope.h): the same names, argument marshalling only.

Every step of the DOPE iteration runs in the library's HIP kernels.  Loading fails loudly when the library
has not been built; there is no CPU fallback."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdope.so")

DOPE_OK = 0
DOPE_EINVAL = -1
DOPE_ENOMEM = -2
DOPE_EDEVICE = -3
DOPE_ENOTSUBMODULAR = -4
DOPE_EOVERFLOW = -5
DOPE_ESOLVER = -6
DOPE_ESTATE = -7
DOPE_EBUSY = -8
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTSUBMODULAR", -5: "EOVERFLOW",
                -6: "ESOLVER", -7: "ESTATE", -8: "EBUSY"}

DOPE_SOLVER_AUTO = 0
DOPE_SOLVER_MAXFLOW = 1
DOPE_SOLVER_EXHAUSTIVE = 2
DOPE_SOLVER_LSATR = 3
DOPE_MEM_HOST = 0
DOPE_MEM_DEVICE = 1


class dope_params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dims", ctypes.c_int32 * 3), ("connectivity", ctypes.c_int32),
                ("block", ctypes.c_int32 * 3), ("overlap", ctypes.c_int32 * 3), ("mu0", ctypes.c_int64),
                ("mu_fact_num", ctypes.c_int32), ("mu_fact_den", ctypes.c_int32), ("eps_q16", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("solver", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class dope_server_params(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int32), ("iters_per_step", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class dope_ml_info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("moves", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("binary_iterations", ctypes.c_int32), ("energy", ctypes.c_int64)]


class dope_info(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int32), ("converged", ctypes.c_int32), ("max_resid2", ctypes.c_int64),
                ("mu", ctypes.c_int64)]


_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_U8P = ctypes.POINTER(ctypes.c_uint8)
_DP = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); the exported C-ABI surface of include/dope.h
SIGNATURES = {
    "dope_create": (ctypes.c_int, [ctypes.POINTER(dope_params), ctypes.POINTER(_P)]),
    "dope_set_energy": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32]),
    "dope_set_energy_async": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32]),
    "dope_iterate": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(dope_info)]),
    "dope_solve": (ctypes.c_int, [_P, ctypes.POINTER(dope_info)]),
    "dope_labels": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "dope_energy": (ctypes.c_int, [_P, _I64P]),
    "dope_get_state": (ctypes.c_int, [_P, _P, _P, _P, _I64P, _I32P]),
    "dope_set_state": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32]),
    "dope_block_resid": (ctypes.c_int, [_P, _P]),
    "dope_block_stats": (ctypes.c_int, [_P, _P]),
    "dope_block_table": (ctypes.c_int, [_P, _I32P, _P]),
    "dope_sizes": (ctypes.c_int, [_P, _I64P, _I32P, _I64P, _I32P]),
    "dope_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(dope_params)]),
    "dope_dispatch_order": (ctypes.c_int, [ctypes.POINTER(dope_params), _I32P, _P]),
    "dope_autotune": (ctypes.c_int, [ctypes.c_int32, _I32P, ctypes.c_int32, _I32P, _I32P]),
    "dope_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "dope_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "dope_profile_read": (ctypes.c_int, [_P, _DP, _I32P, _DP, _I32P]),
    "dope_last_error": (ctypes.c_char_p, [_P]),
    "dope_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P)]),
    "dope_batch_set_energy_async": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _I32P, ctypes.c_int32]),
    "dope_batch_labels": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.c_int32]),
    "dope_batch_iterate": (ctypes.c_int, [_P, ctypes.c_int32]),
    "dope_batch_solve": (ctypes.c_int, [_P]),
    "dope_batch_set_graph": (ctypes.c_int, [_P, ctypes.c_int32]),
    "dope_batch_set_workers": (ctypes.c_int, [_P, ctypes.c_int32]),
    "dope_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(dope_info)]),
    "dope_batch_last_error": (ctypes.c_char_p, [_P]),
    "dope_batch_destroy": (None, [_P]),
    "dope_server_create": (ctypes.c_int, [ctypes.POINTER(dope_server_params), ctypes.POINTER(_P)]),
    "dope_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(dope_params), _P, _P, ctypes.c_int32, ctypes.c_int32,
                                          _P, ctypes.c_int32, _I64P]),
    "dope_server_step": (ctypes.c_int, [_P, _I64P, ctypes.c_int32, _I32P]),
    "dope_server_result": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(dope_info), _I32P]),
    "dope_server_load": (ctypes.c_int, [_P, _I32P, _I32P, ctypes.POINTER(ctypes.c_size_t)]),
    "dope_server_last_error": (ctypes.c_char_p, [_P]),
    "dope_server_destroy": (None, [_P]),
    "dope_solve_noalloc": (ctypes.c_int, [ctypes.POINTER(dope_params), _P, _P, ctypes.c_int32, _P,
                                          ctypes.POINTER(dope_info)]),
    "dope_measure_lds_bandwidth": (ctypes.c_int, [_P, ctypes.c_int32, _DP]),
    "dope_ml_create": (ctypes.c_int, [ctypes.POINTER(dope_params), ctypes.c_int32, ctypes.POINTER(_P)]),
    "dope_ml_set_energy": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "dope_ml_step": (ctypes.c_int, [_P, ctypes.c_int32, _I32P, _I64P]),
    "dope_ml_solve": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(dope_ml_info)]),
    "dope_ml_labels": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "dope_ml_info_get": (ctypes.c_int, [_P, ctypes.POINTER(dope_ml_info)]),
    "dope_ml_last_error": (ctypes.c_char_p, [_P]),
    "dope_ml_destroy": (None, [_P]),
    "dope_destroy": (None, [_P]),
}

DOPE_NOALLOC_MAX_BYTES = 64 << 20

_lib = None


def lib():
    """Load libdope.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                              " (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DopeError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status, ctx=None):
    if status != DOPE_OK:
        msg = lib().dope_last_error(ctx)
        raise DopeError(status, msg.decode() if msg else "")
    return status


def _fn(name):
    def call(*args):
        return getattr(lib(), name)(*args)
    call.__name__ = name
    call.__doc__ = f"C-ABI entry point {name} of include/dope.h"
    return call


dope_create = _fn("dope_create")
dope_set_energy = _fn("dope_set_energy")
dope_set_energy_async = _fn("dope_set_energy_async")
dope_iterate = _fn("dope_iterate")
dope_solve = _fn("dope_solve")
dope_labels = _fn("dope_labels")
dope_energy = _fn("dope_energy")
dope_get_state = _fn("dope_get_state")
dope_set_state = _fn("dope_set_state")
dope_block_resid = _fn("dope_block_resid")
dope_block_stats = _fn("dope_block_stats")
dope_block_table = _fn("dope_block_table")
dope_sizes = _fn("dope_sizes")
dope_workspace_bytes = _fn("dope_workspace_bytes")
dope_dispatch_order = _fn("dope_dispatch_order")
dope_autotune = _fn("dope_autotune")
dope_bind_workspace = _fn("dope_bind_workspace")
dope_profile_enable = _fn("dope_profile_enable")
dope_profile_read = _fn("dope_profile_read")
dope_last_error = _fn("dope_last_error")
dope_destroy = _fn("dope_destroy")
dope_solve_noalloc = _fn("dope_solve_noalloc")
dope_measure_lds_bandwidth = _fn("dope_measure_lds_bandwidth")
dope_ml_create = _fn("dope_ml_create")
dope_ml_set_energy = _fn("dope_ml_set_energy")
dope_ml_step = _fn("dope_ml_step")
dope_ml_solve = _fn("dope_ml_solve")
dope_ml_labels = _fn("dope_ml_labels")
dope_ml_info_get = _fn("dope_ml_info_get")
dope_ml_last_error = _fn("dope_ml_last_error")
dope_ml_destroy = _fn("dope_ml_destroy")
dope_batch_create = _fn("dope_batch_create")
dope_batch_set_energy_async = _fn("dope_batch_set_energy_async")
dope_batch_labels = _fn("dope_batch_labels")
dope_batch_iterate = _fn("dope_batch_iterate")
dope_batch_solve = _fn("dope_batch_solve")
dope_batch_set_graph = _fn("dope_batch_set_graph")
dope_batch_set_workers = _fn("dope_batch_set_workers")
dope_batch_info = _fn("dope_batch_info")
dope_batch_last_error = _fn("dope_batch_last_error")
dope_batch_destroy = _fn("dope_batch_destroy")
dope_server_create = _fn("dope_server_create")
dope_server_submit = _fn("dope_server_submit")
dope_server_step = _fn("dope_server_step")
dope_server_result = _fn("dope_server_result")
dope_server_load = _fn("dope_server_load")
dope_server_last_error = _fn("dope_server_last_error")
dope_server_destroy = _fn("dope_server_destroy")
