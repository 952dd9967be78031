"""ctypes view of libtt.so (the C ABI declared in include/tt.h)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtt.so")

TT_OK = 0
TT_EINVAL = -1
TT_EHIP = -2


class TTGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("coord", ctypes.c_int32),
                ("o", ctypes.c_double * 3), ("h", ctypes.c_double * 3)]


class TTOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("kappa", ctypes.c_double),
                ("tile_k", ctypes.c_int32), ("flags", ctypes.c_int32), ("eps_hist", ctypes.c_void_p)]


EXPORTS = ["tt_workspace_size", "tt_source_params", "tt_forward", "tt_sample", "tt_misfit", "tt_adjoint",
           "tt_kernel", "tt_sweep_timing", "tt_last_error"]

TT_FLAG_TIME_SWEEPS = 1
TT_FLAG_GRAPH = 2

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load(path=LIB_PATH):
    """Load libtt.so.  Raises LibraryMissing if it has not been built: there is
    no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} not found: build it with paper_2412_00031_amd/build.py "
                             "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    G = ctypes.POINTER(TTGrid)
    O = ctypes.POINTER(TTOpts)
    i32 = ctypes.c_int32
    sz = ctypes.c_size_t
    lib.tt_workspace_size.argtypes = [G, i32, O, i32]
    lib.tt_workspace_size.restype = sz
    lib.tt_source_params.argtypes = [G, P, P, P, i32, P, P, P]
    lib.tt_forward.argtypes = [G, P, P, P, i32, P, P, P, O, P, P, P, sz, P]
    lib.tt_sample.argtypes = [G, i32, P, P, P, i32, P, P, P, sz, P]
    lib.tt_misfit.argtypes = [i32, i32, P, P, P, i32, P, P, ctypes.c_double, ctypes.c_double, P, P, P]
    lib.tt_adjoint.argtypes = [G, P, P, P, i32, P, P, P, i32, P, P, O, P, P, P, sz, P]
    lib.tt_kernel.argtypes = [G, P, P, P, i32, P, P, P, P, P, i32, P, sz, P]
    lib.tt_sweep_timing.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32]
    lib.tt_sweep_timing.restype = ctypes.c_int
    lib.tt_last_error.argtypes = []
    lib.tt_last_error.restype = ctypes.c_char_p
    for name in ("tt_source_params", "tt_forward", "tt_sample", "tt_misfit", "tt_adjoint", "tt_kernel"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtt error {code}: {msg}")
        self.code = code


def check(rc):
    if rc != TT_OK:
        raise TTError(rc, load().tt_last_error().decode())
