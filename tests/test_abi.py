"""The C-ABI library loads without a GPU and exports every function that
include/*.h declares (no compute calls)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for fn in sorted(os.listdir(INCLUDE)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"#[^\n]*", "", text)
        for m in re.finditer(r"\b(?:int|int32_t|size_t|void|const\s+char\s*\*)\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def libpath():
    from paper_2412_00031_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.LIB_PATH


def test_headers_declare_the_entry_points():
    names = declared_functions()
    for n in ("tt_forward", "tt_adjoint", "tt_kernel", "tt_sample", "tt_misfit", "tt_workspace_size",
              "tt_last_error", "nn_unet_forward", "nn_unet_backward", "nn_warm_init"):
        assert n in names, n


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert declared_functions() <= exported


def test_binding_declares_every_header_symbol():
    from paper_2412_00031_amd import _lib
    assert declared_functions() == set(_lib.EXPORTS) | set(_lib.NN_EXPORTS)


def test_binding_constants_match_the_header():
    """Every TT_* integer constant of include/tt.h has the same value in the binding."""
    from paper_2412_00031_amd import _lib
    text = open(os.path.join(INCLUDE, "tt.h")).read()
    defs = dict(re.findall(r"#define\s+(TT_[A-Z0-9_]+)\s+(-?\d+)\b", text))
    assert {"TT_FLAG_POLL", "TT_FLAG_COMPACT_ADJOINT", "TT_FLAG_ADJOINT_INIT"} <= set(defs)
    for name, v in defs.items():
        if hasattr(_lib, name):
            assert getattr(_lib, name) == int(v), name
    flags = [int(v) for k, v in defs.items() if k.startswith("TT_FLAG_")]
    assert len(set(flags)) == len(flags) and all(f & (f - 1) == 0 for f in flags)


def test_last_error_without_gpu(libpath):
    """A host-checked argument error is reported without touching a device."""
    from paper_2412_00031_amd import _lib
    lib = _lib.load(libpath)
    rc = lib.tt_misfit(0, 1, None, None, None, 0, None, None, 1.0, 1.0, None, None, None)
    assert rc == _lib.TT_EINVAL
    assert lib.tt_last_error().decode()


def test_mg_workspace_size_host_logic(libpath):
    """The projection's plan is host logic: staged (with workspace) for the
    benchmark's five 11 x 13 x 13 grids on 101^3, one wave per node (no
    workspace) when the staging exceeds LDS, 0 for invalid sizes."""
    from paper_2412_00031_amd import _lib, api, workloads as W
    _lib.load(libpath)
    g = W.spherical_grid(101, 100.0, 2.0)
    inv = W.staggered_inversion_grids(g, (11, 13, 13), 5)
    nb = api.mg_workspace_size(g, inv)
    S12 = 5 * 13 * 13
    assert nb > 0 and nb % (8 * 101 * 3 * S12) == 0 and nb // (8 * 101 * 3 * S12) <= 8
    big = [(np.zeros(5), np.zeros(70), np.zeros(70))] * 2
    assert api.mg_workspace_size(g, big) == 0
    assert api.mg_workspace_size(g, [(np.zeros(0), np.zeros(2), np.zeros(2))]) == 0
    assert api.mg_workspace_size(g, [(np.zeros(2), np.zeros(2), np.zeros(2))] * 17) == 0


def test_workspace_sizes_host_logic(libpath):
    """Workspace sizing is host logic: an empty batch needs zero bytes, every
    non-empty one a positive size that grows with the batch, and a bad tile
    depth or source count is refused (size 0 -> ValueError in the binding)."""
    from paper_2412_00031_amd import _lib, api, workloads as W
    _lib.load(libpath)
    g = W.spherical_grid(21, 20.0, 2.0)
    for which in range(4):
        assert api.workspace(g, 0, which).numel() == 0
        a, b = api.workspace(g, 1, which).numel(), api.workspace(g, 5, which).numel()
        assert 0 < a <= b
    with pytest.raises(ValueError):
        api.workspace(g, 1, 0, tile_k=63)
    # the compact adjoint records take one node-order copy instead of four row layouts
    fast, compact = api.workspace(g, 3, 1).numel(), api.workspace(g, 3, 1, compact=True).numel()
    assert 0 < compact < fast
    with pytest.raises(ValueError):
        api.workspace(g, -1, 1)


def test_grid_size_limit_uses_the_record_pitch(libpath):
    """Records are addressed with 32-bit indices within one layout of
    n0 (n1 + n2 - 1) n1p records (n1p = n1 + 7 rounded up to 8), so the grid
    check bounds that product, not n0 (n1 + n2 - 1) n1: (8192, 31, 8192) has
    2.09e9 < 2^31 unpadded but 2.69e9 padded records."""
    import ctypes
    from paper_2412_00031_amd import _lib, api
    lib = _lib.load(libpath)

    def size(n):
        g = dict(n=n, coord=0, o=(0.0, 0.0, 0.0), h=(1.0, 1.0, 1.0))
        return lib.tt_workspace_size(ctypes.byref(api._grid(g)), 1, None, 0)

    assert size((8192, 31, 8192)) == 0
    assert size((8192, 20, 8192)) == 0      # 1.35e9 unpadded, 2.15e9 padded (n1p = 32)
    assert size((8192, 9, 8192)) > 0        # 1.07e9 padded (n1p = 16)
    assert size((4096, 31, 4096)) > 0
    assert size((101, 101, 101)) > 0


def test_tune_cache_key_names_build_and_device(libpath, monkeypatch):
    """Tile-depth choices are cached per (kind, grid, source count, library
    build, device): a rebuilt library must not reuse choices measured on
    another build."""
    from paper_2412_00031_amd import _lib, autotune, workloads as W
    _lib.load(libpath)
    g = W.spherical_grid(21, 20.0, 2.0)
    k1 = autotune._key("fwd", g, 8)
    assert _lib.build_id() in k1 and k1 != autotune._key("adj", g, 8) and k1 != autotune._key("fwd", g, 9)
    monkeypatch.setattr(_lib, "_build_id", "0" * 16)
    assert autotune._key("fwd", g, 8) != k1


def test_default_tile_depths_exported(libpath):
    """tile_k = 0 selects the depths the library exports (one shared place for
    the bench's labels and traffic lookups)."""
    from paper_2412_00031_amd import _lib
    lib = _lib.load()
    assert 1 <= lib.tt_default_tile_k(0) <= 62 and 1 <= lib.tt_default_tile_k(1) <= 62
    assert lib.tt_default_tile_k(2) == 0


def test_budget_marshalling_host_logic():
    """Per-source iteration budgets are marshalled as a host int32 array of
    one entry per source (lists, numpy arrays and CPU tensors alike); a wrong
    length is refused before any library call; the options struct carries its
    address."""
    import torch
    from paper_2412_00031_amd import api
    b = api._budgets([3, 4, 5], 3)
    assert b.dtype == np.int32 and b.tolist() == [3, 4, 5] and b.flags["C_CONTIGUOUS"]
    assert api._budgets(torch.tensor([7, 8], dtype=torch.int64), 2).tolist() == [7, 8]
    assert api._budgets(None, 4) is None
    with pytest.raises(ValueError):
        api._budgets([1, 2], 3)
    o = api._opts(1e-6, 10, 1.0, budgets=b)
    assert o.budgets == b.ctypes.data and o.max_iter == 10
    assert api._opts(1e-6, 10, 1.0).budgets is None
