"""Autotuner for the sweep launch shape of the forward and adjoint solves:
the tile depth (tile_k, the hyperplane steps of one sweep tile) and the
number of concurrently iterated source groups.

For a grid and source count it times a few iterations of each solve for every
candidate tile depth (the whole call, asynchronous as in production, with the
library's default source groups), on the whole batch and on a quarter of it
(the convergence tail of a solve runs with few sources left), keeps the
fastest sum, and then times the source-group counts at that depth.  Every
fixed-iteration candidate is timed over exactly the requested iterations: the
tolerance is unreachable and the statuses are checked afterwards (a candidate
that stopped early would look fast).

With a tolerance (``tol``) the group counts are timed on whole solves of the
batch to that tolerance instead: asynchronous, with per-source budgets from a
host-polled solve (each source's iteration count plus a margin), every status
checked.  Groups matter most in the convergence tail, when each group's
launches carry a few sources and the groups fill each other's idle units, and
a few iterations of the whole batch do not show that.

Any tile depth and any grouping give bit-identical results, so the choice
affects speed only.  Choices are cached in a JSON file keyed by (kind,
coordinates, grid shape, source count, library build, device name, hardware
queues, tuning mode), so a rebuilt library is tuned afresh; the file is
``$TT_TUNE_CACHE`` or ``~/.cache/paper_2412_00031_amd/tiles.json``.
"""
import json
import os

import torch

from . import _lib, api

CANDIDATES = (8, 12, 14, 16, 18, 20, 22, 24, 28, 32, 40, 48, 62)
GROUP_CANDIDATES = (1, 2, 3, 4, 6, 8)


def cache_path():
    p = os.environ.get("TT_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2412_00031_amd", "tiles.json")


def _key(kind, grid, nsrc, tol=None):
    n = "x".join(str(int(v)) for v in grid["n"])
    dev = torch.cuda.get_device_name().replace(":", " ") if torch.cuda.is_available() else "none"
    hwq = os.environ.get("GPU_MAX_HW_QUEUES", "default")
    mode = "iters" if tol is None else f"tol{tol:g}"
    return f"{kind}:{int(grid['coord'])}:{n}:{int(nsrc)}:{_lib.build_id()}:{dev}:hwq{hwq}:{mode}"


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


def _elapsed_ms(fn, iters):
    """Device time of one call of fn (HIP events on the current stream, which
    the binding hands to the library), after checking that every source ran
    all `iters` iterations."""
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, st = fn()
    e1.record()
    torch.cuda.synchronize()
    if not bool((st == -iters).all()):
        raise RuntimeError(f"autotune: a timed solve did not run its {iters} iterations (statuses "
                           f"{st.min().item()}..{st.max().item()}); its timing would be meaningless")
    return e0.elapsed_time(e1)


def _time(kind, grid, s, xi, eta, src, par, tau, rec, R, kappa, tk, groups, iters):
    if kind == "fwd":
        return _elapsed_ms(lambda: api.forward(grid, s, xi, eta, src, par, 1e-300, iters, kappa, tile_k=tk,
                                               groups=groups), iters)
    return _elapsed_ms(lambda: api.adjoint(grid, s, xi, eta, src, par, tau, rec, R, 1e-300, iters, kappa, tile_k=tk,
                                           groups=groups), iters)


BUDGET_MARGIN = 8


def _solve(kind, grid, s, xi, eta, src, par, tau, rec, R, kappa, tol, max_iter, tk, groups, poll=False,
           budgets=None):
    if kind == "fwd":
        return api.forward(grid, s, xi, eta, src, par, tol, max_iter, kappa, tile_k=tk, groups=groups, poll=poll,
                           budgets=budgets)
    return api.adjoint(grid, s, xi, eta, src, par, tau, rec, R, tol, max_iter, kappa, tile_k=tk, groups=groups,
                       poll=poll, budgets=budgets)


def _converged_ms(kind, grid, s, xi, eta, src, par, tau, rec, R, kappa, tol, budgets, tk, groups):
    """Device time of a whole asynchronous solve to tol within per-source
    iteration budgets; every source must converge."""
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, st = _solve(kind, grid, s, xi, eta, src, par, tau, rec, R, kappa, tol, int(budgets.max()), tk, groups,
                   budgets=budgets)
    e1.record()
    torch.cuda.synchronize()
    if not bool((st > 0).all()):
        raise RuntimeError(f"autotune: a {kind} solve did not converge within its iteration budgets")
    return e0.elapsed_time(e1)


def tune(grid, s, xi, eta, src, par, kappa, rec, R=None, iters=3, candidates=CANDIDATES,
         group_candidates=GROUP_CANDIDATES, use_cache=True, log=None, tol=None):
    """Return {"fwd": tile_k, "adj": tile_k, "groups_fwd": g, "groups_adj": g}
    for this grid and batch size.  R: the adjoint sources the adjoint solves
    are timed with (any nonzero values; default all ones).  tol: time the
    group counts on whole solves to this tolerance (see the module notes)."""
    nsrc = int(src.shape[0])
    cache = _load() if use_cache else {}
    keys = {kind: _key(kind, grid, nsrc, tol) for kind in ("fwd", "adj")}
    if use_cache and all(k in cache and "groups" in cache[k] for k in keys.values()):
        return {"fwd": int(cache[keys["fwd"]]["tile_k"]), "adj": int(cache[keys["adj"]]["tile_k"]),
                "groups_fwd": int(cache[keys["fwd"]]["groups"]), "groups_adj": int(cache[keys["adj"]]["groups"]),
                "cached": True}
    if R is None:
        R = torch.ones((nsrc, int(rec.shape[0])), dtype=torch.float64, device=s.device)
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
        def cost(tk, groups):
            ms = 0.0
            for (sp, pp, tp, rp) in parts:
                ms += min(_time(kind, grid, s, xi, eta, sp, pp, tp, rec, rp, kappa, tk, groups, iters)
                          for _ in range(2))
            return round(ms, 3)
        times = {tk: cost(tk, 0) for tk in cands}
        best = min(times, key=times.get)
        gcands = [gq for gq in group_candidates if gq <= max(1, nsrc)]
        if tol is None:
            gtimes = {gq: cost(best, gq) for gq in gcands}
        else:
            # whole solves to tol: the forward from tau = 1, the adjoint at the
            # converged forward field
            tau_c = None
            if kind == "adj":
                tau_c, _ = _solve("fwd", grid, s, xi, eta, src, par, None, rec, R, kappa, tol, 1000, res["fwd"], 0,
                                  poll=True)
            _, st_p = _solve(kind, grid, s, xi, eta, src, par, tau_c, rec, R, kappa, tol, 1000, best, 0, poll=True)
            if not bool((st_p > 0).all()):
                raise RuntimeError(f"autotune: a host-polled {kind} solve did not converge in 1000 iterations")
            budgets = st_p.cpu().numpy() + BUDGET_MARGIN
            gtimes = {gq: round(min(_converged_ms(kind, grid, s, xi, eta, src, par, tau_c, rec, R, kappa, tol,
                                                  budgets, best, gq) for _ in range(2)), 3) for gq in gcands}
        bestg = min(gtimes, key=gtimes.get)
        res[kind] = best
        res["groups_" + kind] = bestg
        cache[keys[kind]] = {"tile_k": best, "groups": bestg, "ms": times, "groups_ms": gtimes}
        if log:
            log(f"autotune {kind}: tile_k {best} ({times}); groups {bestg} ({gtimes})")
    if use_cache:
        _store(cache)
    res["cached"] = False
    return res
