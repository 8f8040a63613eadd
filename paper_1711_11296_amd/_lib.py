"""ctypes binding of libsht.so (argument marshalling only).

The library is loaded after torch so that both share the one HIP runtime of
the process.  There is no fallback: if the library is missing, loading fails
with an error that says how to build it.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsht.so")

GRID = {"cc_poles": 0, "fejer2": 1, "fejer1": 2, "gauss": 3}
FORM = {"fp64": 0, "fp32": 1, "bf16x6": 2}

SHT_OK, SHT_EINVAL, SHT_ENOMEM, SHT_EHIP, SHT_ESTATE = 0, -1, -2, -3, -4
Q_NLEVELS, Q_NCOEF, Q_EXACT, Q_WORKSPACE_BYTES, Q_TABLE_BYTES = 0, 1, 2, 3, 4
Q_GRID_ELEMS, Q_SPEC_ELEMS, Q_FORM, Q_GRID_KIND, Q_LEGENDRE_FLOPS = 5, 6, 7, 8, 9
Q_LEGENDRE_FLOPS_KEPT = 10
Q_ZONAL_ONE_LAUNCH = 11
Q_GRID_OFFSET, Q_SPEC_OFFSET = 100, 200

EXPORTS = ["sht_plan", "sht_plan_ex", "sht_plan_multi", "sht_forward", "sht_inverse",
           "sht_forward_adjoint", "sht_inverse_adjoint", "sht_plan_query",
           "sht_plan_tables", "sht_plan_destroy", "sht_last_error", "sht_host_tables",
           "sht_plan_profile", "sht_plan_profile_read", "sht_spec_retruncate", "sht_grid_inject",
           "sht_grid_product", "sht_spec_laplacian", "sht_grid_residual", "sht_device_bytes",
           "sht_forward_noalloc"]


class SHTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sht error %d: %s" % (code, msg))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int), ("form", ctypes.c_int),
                ("autotune", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("reduced", ctypes.c_int), ("otf", ctypes.c_int), ("zonal", ctypes.c_int)]


ZONAL = {"auto": 0, "one_launch": 1, "per_length": 2}


_lib = None


def load(require_torch=True):
    """Load libsht.so (importing torch first unless require_torch=False,
    which is only meant for host-only entry points)."""
    global _lib
    if _lib is not None:
        return _lib
    if require_torch:
        import torch  # noqa: F401  (one HIP runtime per process)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsht.so is not built; run `python -c \"import __graft_entry__ as g; g.build()\"` "
                           "or `python paper_1711_11296_amd/_build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, c_int = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.sht_plan.restype = vp
    lib.sht_plan.argtypes = [c_int, c_int, c_int, c_int]
    lib.sht_plan_ex.restype = c_int
    lib.sht_plan_ex.argtypes = [c_int, c_int, c_int, c_int, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.sht_plan_multi.restype = c_int
    lib.sht_plan_multi.argtypes = [c_int, ip, ip, ip, ip, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    for name in ("sht_forward", "sht_inverse", "sht_forward_adjoint", "sht_inverse_adjoint", "sht_forward_noalloc"):
        f = getattr(lib, name)
        f.restype = c_int
        f.argtypes = [vp, vp, vp, vp]
    lib.sht_plan_query.restype = c_int
    lib.sht_plan_query.argtypes = [vp, c_int, vp]
    lib.sht_plan_tables.restype = c_int
    lib.sht_plan_tables.argtypes = [vp, dp, dp, dp]
    lib.sht_plan_destroy.restype = c_int
    lib.sht_plan_destroy.argtypes = [vp]
    lib.sht_last_error.restype = ctypes.c_char_p
    lib.sht_last_error.argtypes = []
    lib.sht_plan_profile.restype = c_int
    lib.sht_plan_profile.argtypes = [vp, c_int]
    lib.sht_plan_profile_read.restype = c_int
    lib.sht_plan_profile_read.argtypes = [vp, dp, ip]
    lib.sht_spec_retruncate.restype = c_int
    lib.sht_spec_retruncate.argtypes = [c_int, c_int, c_int, c_int, vp, vp, vp]
    lib.sht_grid_product.restype = c_int
    lib.sht_grid_product.argtypes = [ctypes.c_longlong, c_int, vp, vp, vp, vp]
    lib.sht_spec_laplacian.restype = c_int
    lib.sht_spec_laplacian.argtypes = [c_int, c_int, c_int, ctypes.c_double, vp, vp, vp]
    lib.sht_grid_residual.restype = c_int
    lib.sht_grid_residual.argtypes = [ctypes.c_longlong, ctypes.c_longlong, c_int, ctypes.c_double,
                                      vp, vp, vp, vp, vp, vp]
    lib.sht_grid_inject.restype = c_int
    lib.sht_grid_inject.argtypes = [c_int, c_int, c_int, c_int, c_int, c_int, c_int, vp, vp, vp]
    lib.sht_host_tables.restype = c_int
    lib.sht_host_tables.argtypes = [c_int, c_int, c_int, dp, dp, dp]
    lib.sht_device_bytes.restype = c_int
    lib.sht_device_bytes.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
    _lib = lib
    return lib


def check(rc):
    if rc != SHT_OK:
        raise SHTError(rc, _lib.sht_last_error().decode())
    return rc


def last_error():
    return load(False).sht_last_error().decode()


def device_bytes():
    """Device bytes held by all live plans of the process."""
    lib = load(False)
    v = ctypes.c_size_t(0)
    check(lib.sht_device_bytes(ctypes.byref(v)))
    return int(v.value)
