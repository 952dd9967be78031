"""Evaluation of the learned warm start on the 121^3 workload (sph121, 512
sources): plain and warm-started forward solves to the same tolerance 1e-6,
compared on iteration counts, wall time and final error against a tol-1e-13
solution of a subset of the sources.  The network was trained on the 101^3
geometry (h = 1 km); it is fully convolutional on a stride-2 coarse grid of
physical features, so it runs unchanged at h = 0.83 km.

    python -m paper_2412_00031_amd.eval_warmstart [--nsrc 512] [--ref-sources 32]

prints one JSON object."""
import argparse
import json
import sys
import time

import numpy as np
import torch

from . import api, workloads as W
from .warmstart import WEIGHTS, UNet, WarmStart


def evaluate(nsrc=512, ref_sources=32, weights=WEIGHTS, device="cuda", max_iter=20000, log=print):
    wl = W.sph121(nsrc=nsrc)
    g, kappa, tol = wl["grid"], wl["kappa"], wl["tol"]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
    s, xi, eta, src = dev(wl["s"]), dev(wl["xi"]), dev(wl["eta"]), dev(wl["src"])
    par = api.source_params(g, s, xi, eta, src)
    warm = WarmStart(UNet.load(weights, device), g)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    (tau_p, st_p), t_p = timed(lambda: api.forward(g, s, xi, eta, src, par, tol, max_iter, kappa, poll=True))
    log(f"plain: {t_p:.2f} s")
    init, t_pred = timed(lambda: warm.predict(s, xi, eta, src, par))
    (tau_w, st_w), t_w = timed(lambda: api.forward(g, s, xi, eta, src, par, tol, max_iter, kappa, tau_init=init, poll=True))
    log(f"warm: {t_pred:.2f} s prediction + {t_w:.2f} s sweeps")
    q = min(ref_sources, nsrc)
    tau_r, st_r = api.forward(g, s, xi, eta, src[:q], par[:q], 1e-13, max_iter, kappa, poll=True)
    ip, iw, ir = (x.cpu().numpy() for x in (st_p, st_w, st_r))
    if (ip <= 0).any() or (iw <= 0).any() or (ir <= 0).any():
        raise RuntimeError("a solve did not converge")
    e_p = (tau_p[:q] - tau_r).abs().flatten(1)
    e_w = (tau_w[:q] - tau_r).abs().flatten(1)
    e_i = (init.view_as(tau_w)[:q] - tau_r).abs().flatten(1)
    e_1 = (1.0 - tau_r).abs().flatten(1)
    return {
        "workload": f"sph121: 121^3 spherical (0-100 km, 4x4 deg), GRF model, {nsrc} sources, tol {tol:g}",
        "plain": {"mean_iters": round(float(ip.mean()), 2), "max_iters": int(ip.max()), "forward_s": round(t_p, 3)},
        "warm": {"mean_iters": round(float(iw.mean()), 2), "max_iters": int(iw.max()), "forward_s": round(t_w, 3),
                 "predict_s": round(t_pred, 3)},
        "iteration_ratio": round(float(iw.sum() / ip.sum()), 4),
        "final_error_vs_tol_1e-13": {"sources": q, "plain_max": float(e_p.max()), "warm_max": float(e_w.max()),
                                     "plain_mean": float(e_p.mean()), "warm_mean": float(e_w.mean())},
        "initial_error_mean": {"plain": float(e_1.mean()), "warm": float(e_i.mean())},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsrc", type=int, default=512)
    ap.add_argument("--ref-sources", type=int, default=32)
    ap.add_argument("--weights", default=WEIGHTS)
    a = ap.parse_args()
    res = evaluate(a.nsrc, a.ref_sources, a.weights, log=lambda m: print(f"[eval] {m}", file=sys.stderr, flush=True))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
