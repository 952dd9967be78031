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
                ("tile_k", ctypes.c_int32), ("flags", ctypes.c_int32), ("eps_hist", ctypes.c_void_p),
                ("groups", ctypes.c_int32), ("budgets", ctypes.c_void_p)]


EXPORTS = ["tt_workspace_size", "tt_source_params", "tt_forward", "tt_forward_noalloc", "tt_forward_noalloc_limit", "tt_sample", "tt_misfit", "tt_misfit_cr", "tt_reloc_times", "tt_reloc_kernel",
           "tt_adjoint", "tt_kernel", "tt_kernel_density", "tt_mg_workspace_size", "tt_mg_project", "tt_mg_expand",
           "tt_sweep_timing", "tt_default_tile_k", "tt_last_error"]

NN_EXPORTS = ["nn_to_bf16", "nn_from_bf16", "nn_conv3_pack", "nn_conv3_fwd", "nn_conv3_wgrad_work", "nn_conv3_wgrad",
              "nn_relu_mask", "nn_pool_fwd", "nn_pool_bwd", "nn_up_fwd", "nn_up_wgrad_work", "nn_up_bwd",
              "nn_head_fwd", "nn_head_work", "nn_head_bwd", "nn_mse", "nn_adam", "nn_unet_nparams", "nn_unet_nfrag",
              "nn_unet_workspace", "nn_unet_pack", "nn_unet_forward", "nn_unet_backward", "nn_warm_features",
              "nn_warm_target", "nn_warm_init"]

# constants of include/nn.h
NN_FEAT_S = 5.0
NN_FEAT_A = 25.0
NN_FEAT_D = 0.01
NN_TARGET_SCALE = 10.0
NN_MSE_LOSS_FLOATS = 2 + 2 * 1024


class NNUnetCfg(ctypes.Structure):
    _fields_ = [("ch", ctypes.c_int32 * 4), ("in_ch", ctypes.c_int32)]

TT_FLAG_TIME_SWEEPS = 1
TT_FLAG_GRAPH = 2
TT_FLAG_CONTINUOUS_ADJOINT = 4
TT_FLAG_POLL = 8
TT_FLAG_COMPACT_ADJOINT = 16
TT_FLAG_ADJOINT_INIT = 32
TT_ENOCONV = -3
TT_MAX_GROUPS = 8

_lib = None


class LibraryMissing(RuntimeError):
    pass


_lib_path = None
_build_id = None


def build_id():
    """Short sha256 of the loaded library file: identifies the build (tile-depth
    choices measured on one build are not reused for another)."""
    global _build_id
    if _build_id is None:
        import hashlib
        load()
        with open(_lib_path, "rb") as f:
            _build_id = hashlib.sha256(f.read()).hexdigest()[:16]
    return _build_id


def load(path=LIB_PATH):
    """Load libtt.so.  Raises LibraryMissing if it has not been built: there is
    no fallback implementation."""
    global _lib, _lib_path
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} not found: build it with `python -m paper_2412_00031_amd.build`; "
                             "there is no CPU fallback")
    lib = ctypes.CDLL(path)
    _lib_path = path
    P = ctypes.c_void_p
    G = ctypes.POINTER(TTGrid)
    O = ctypes.POINTER(TTOpts)
    i32 = ctypes.c_int32
    sz = ctypes.c_size_t
    lib.tt_workspace_size.argtypes = [G, i32, O, i32]
    lib.tt_workspace_size.restype = sz
    lib.tt_source_params.argtypes = [G, P, P, P, i32, P, P, P]
    lib.tt_forward.argtypes = [G, P, P, P, i32, P, P, P, O, P, P, P, sz, P]
    lib.tt_forward_noalloc.argtypes = [G, P, P, P, i32, P, P, P, O, P, P, P]
    lib.tt_forward_noalloc_limit.argtypes = []
    lib.tt_forward_noalloc_limit.restype = sz
    lib.tt_sample.argtypes = [G, i32, P, P, P, i32, P, P, P, sz, P]
    lib.tt_misfit.argtypes = [i32, i32, P, P, P, i32, P, P, ctypes.c_double, ctypes.c_double, P, P, P]
    lib.tt_reloc_times.argtypes = [G, i32, P, P, P, i32, P, P, P, P, sz, P]
    lib.tt_reloc_kernel.argtypes = [G, i32, P, P, P, i32, P, P, P, P, sz, P]
    lib.tt_misfit_cr.argtypes = [i32, i32, P, P, P, P, P, ctypes.c_double, P, P, P]
    lib.tt_adjoint.argtypes = [G, P, P, P, i32, P, P, P, i32, P, P, O, P, P, P, sz, P]
    lib.tt_kernel.argtypes = [G, P, P, P, i32, P, P, P, P, P, i32, P, sz, P]
    lib.tt_kernel_density.argtypes = [G, P, P, P, ctypes.c_double, ctypes.c_double, P, P, P]
    lib.tt_mg_workspace_size.argtypes = [G, i32, ctypes.POINTER(i32)]
    lib.tt_mg_workspace_size.restype = sz
    lib.tt_mg_project.argtypes = [G, i32, ctypes.POINTER(i32), P, P, P, P, sz, P]
    lib.tt_mg_expand.argtypes = [G, i32, ctypes.POINTER(i32), P, P, P, P]
    lib.tt_sweep_timing.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32]
    lib.tt_sweep_timing.restype = ctypes.c_int
    lib.tt_default_tile_k.argtypes = [i32]
    lib.tt_default_tile_k.restype = i32
    lib.tt_last_error.argtypes = []
    lib.tt_last_error.restype = ctypes.c_char_p
    for name in ("tt_source_params", "tt_forward", "tt_forward_noalloc", "tt_sample", "tt_misfit", "tt_misfit_cr", "tt_reloc_times",
                 "tt_reloc_kernel", "tt_adjoint", "tt_kernel", "tt_kernel_density", "tt_mg_project", "tt_mg_expand"):
        getattr(lib, name).restype = ctypes.c_int
    _declare_nn(lib)
    _lib = lib
    return lib


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtt error {code}: {msg}")
        self.code = code


def check(rc):
    if rc != TT_OK:
        raise TTError(rc, load().tt_last_error().decode())


def _declare_nn(lib):
    P = ctypes.c_void_p
    G = ctypes.POINTER(TTGrid)
    C = ctypes.POINTER(NNUnetCfg)
    i = ctypes.c_int
    i64 = ctypes.c_int64
    sz = ctypes.c_size_t
    f = ctypes.c_float
    sig = {
        "nn_to_bf16": [P, i64, P, P],
        "nn_from_bf16": [P, i64, P, P],
        "nn_conv3_pack": [P, i, i, i, P, P],
        "nn_conv3_fwd": [P, i, i, i, i, i, i, i, P, P, i, i, P, i, i, P],
        "nn_conv3_wgrad": [P, i, i, i, i, i, i, i, P, i, i, i, P, P, P, sz, P],
        "nn_relu_mask": [P, P, i64, i, i, i, P, i, i, P],
        "nn_pool_fwd": [P, i, i, i, i, i, i, i, P, P],
        "nn_pool_bwd": [P, P, i, i, i, i, i, i, i, P, i, P],
        "nn_up_fwd": [P, i, i, i, i, i, P, P, i, P, i, i, P],
        "nn_up_bwd": [P, P, i, i, i, i, i, i, i, i, P, P, P, P, P, sz, P],
        "nn_head_fwd": [P, i64, i, P, P, P, P],
        "nn_head_bwd": [P, P, i64, i, P, P, P, P, P, sz, P],
        "nn_mse": [P, P, P, i64, P, P, P],
        "nn_adam": [P, P, P, P, i64, i, f, f, f, f, P],
        "nn_unet_pack": [C, P, P, P],
        "nn_unet_forward": [C, P, P, P, i, i, i, i, P, P, sz, i, P],
        "nn_unet_backward": [C, P, P, P, P, i, i, i, i, P, P, sz, P],
        "nn_warm_features": [G, P, P, P, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_int32, P, P],
        "nn_warm_target": [G, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P,
                           P],
        "nn_warm_init": [G, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    sizes = {
        "nn_conv3_wgrad_work": [i, i, i, i, i, i],
        "nn_up_wgrad_work": [i, i, i, i, i, i],
        "nn_head_work": [i64, i],
        "nn_unet_nparams": [C],
        "nn_unet_nfrag": [C],
        "nn_unet_workspace": [C, i, i, i, i, i],
    }
    for name, args in sizes.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = sz
