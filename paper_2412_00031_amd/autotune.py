"""Autotuner for the sweep tile depth (tile_k) of the forward and adjoint solves.

For a grid and source count it times a few iterations of each solve for every
candidate tile depth (the whole call, with the library's default source groups
running concurrently, as in production), on the whole batch and on a quarter of
it (the convergence tail of a solve runs with few sources left), and keeps the
fastest sum.  Any tile depth gives
bit-identical results, so the choice affects speed only.  Choices are cached in
a JSON file keyed by (kind, coordinates, grid shape, source count, library
build, device name), so a rebuilt library is tuned afresh; the file is
``$TT_TUNE_CACHE`` or ``~/.cache/paper_2412_00031_amd/tiles.json``.
"""
import json
import os

import torch

from . import _lib, api

CANDIDATES = (8, 12, 16, 18, 20, 22, 24, 28, 32, 40, 48, 62)


def cache_path():
    p = os.environ.get("TT_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2412_00031_amd", "tiles.json")


def _key(kind, grid, nsrc):
    n = "x".join(str(int(v)) for v in grid["n"])
    dev = torch.cuda.get_device_name().replace(":", " ") if torch.cuda.is_available() else "none"
    return f"{kind}:{int(grid['coord'])}:{n}:{int(nsrc)}:{_lib.build_id()}:{dev}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


# Each candidate is timed as the solves run in production: the whole call
# (sweeps, boundary passes, convergence checks) with the library's default
# source groups running concurrently, over a fixed iteration count.
def _elapsed_ms(fn):
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _time_fwd(grid, s, xi, eta, src, par, kappa, tk, iters):
    return _elapsed_ms(lambda: api.forward(grid, s, xi, eta, src, par, 1e-300, iters, kappa, tile_k=tk))


def _time_adj(grid, s, xi, eta, src, par, tau, rec, R, kappa, tk, iters):
    return _elapsed_ms(lambda: api.adjoint(grid, s, xi, eta, src, par, tau, rec, R, 1e-300, iters, kappa, tile_k=tk))


def tune(grid, s, xi, eta, src, par, kappa, rec, R, iters=3, candidates=CANDIDATES, use_cache=True, log=None):
    """Return {"fwd": tile_k, "adj": tile_k} for this grid and batch size."""
    nsrc = int(src.shape[0])
    cache = _load() if use_cache else {}
    kf, ka = _key("fwd", grid, nsrc), _key("adj", grid, nsrc)
    if use_cache and kf in cache and ka in cache:
        return {"fwd": int(cache[kf]["tile_k"]), "adj": int(cache[ka]["tile_k"]), "cached": True}
    m2 = int(grid["n"][2]) - 2
    cands = sorted({min(c, m2, 62) for c in candidates})
    tau, _ = api.forward(grid, s, xi, eta, src, par, 1e-300, iters, kappa)
    # a solve runs most iterations with the whole batch active and ends with a
    # tail in which a few sources are left: each candidate is timed on the whole
    # batch and on its first quarter, and the two times are added
    nq = max(1, nsrc // 4)
    parts = [(src, par, tau, R)] + ([(src[:nq], par[:nq], tau[:nq], R[:nq])] if nq < nsrc else [])
    res = {}
    for kind in ("fwd", "adj"):
        best, best_ms, times = None, None, {}
        for tk in cands:
            ms = 0.0
            for (sp, pp, tp, rp) in parts:
                ms += min((_time_fwd(grid, s, xi, eta, sp, pp, kappa, tk, iters) if kind == "fwd" else
                           _time_adj(grid, s, xi, eta, sp, pp, tp, rec, rp, kappa, tk, iters)) for _ in range(2))
            times[tk] = round(ms, 3)
            if best_ms is None or ms < best_ms:
                best, best_ms = tk, ms
        res[kind] = best
        cache[_key(kind, grid, nsrc)] = {"tile_k": best, "ms": times}
        if log:
            log(f"autotune {kind}: tile_k {best} ({times})")
    if use_cache:
        _store(cache)
    res["cached"] = False
    return res
