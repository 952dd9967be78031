"""The learned warm start on the GPU: what the shipped network gains over the
plain start, at equal accuracy, and that a poor prediction costs iterations
but never accuracy (the sweeps always run to the same tolerance)."""
import os

import numpy as np
import pytest

from paper_2412_00031_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setup(torch, nsrc, first=0):
    from paper_2412_00031_amd import api
    wl = W.sph101(with_true=False)  # held out: no training model uses its seeds
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    s, xi, eta = dev(wl["s"]), dev(wl["xi"]), dev(wl["eta"])
    src = dev(wl["src"][first:first + nsrc])
    par = api.source_params(wl["grid"], s, xi, eta, src)
    return wl, s, xi, eta, src, par


def _solve(torch, wl, s, xi, eta, src, par, tol, init=None):
    from paper_2412_00031_amd import api
    return api.forward(wl["grid"], s, xi, eta, src, par, tol, 20000, wl["kappa"], tau_init=init, poll=True)


def test_shipped_network_cuts_sweeps_at_equal_accuracy(torch_cuda):
    """16 sources of the 101^3 workload model (never trained on): the warm
    start needs fewer iterations to tol 1e-6, and its result is as close to the
    tol-1e-13 solution as the plain one."""
    from paper_2412_00031_amd.warmstart import WEIGHTS, UNet, WarmStart
    torch = torch_cuda
    assert os.path.exists(WEIGHTS), WEIGHTS
    wl, s, xi, eta, src, par = _setup(torch, 16)
    ws = WarmStart(UNet.load(WEIGHTS, "cuda"), wl["grid"])
    init = ws.predict(s, xi, eta, src, par)
    tau_p, st_p = _solve(torch, wl, s, xi, eta, src, par, 1e-6)
    tau_w, st_w = _solve(torch, wl, s, xi, eta, src, par, 1e-6, init)
    tau_r, st_r = _solve(torch, wl, s, xi, eta, src, par, 1e-13)
    ip, iw = st_p.cpu().numpy(), st_w.cpu().numpy()
    assert (ip > 0).all() and (iw > 0).all() and (st_r.cpu().numpy() > 0).all()
    init_err = float((init.view_as(tau_r) - tau_r).abs().mean())
    one_err = float((1.0 - tau_r).abs().mean())
    print(f"iterations plain {ip.mean():.2f} warm {iw.mean():.2f}; initial error plain {one_err:.3e} warm "
          f"{init_err:.3e}")
    assert init_err < 0.5 * one_err
    assert iw.mean() < ip.mean()
    assert iw.sum() <= 0.97 * ip.sum()
    e_p = float((tau_p - tau_r).abs().max())
    e_w = float((tau_w - tau_r).abs().max())
    assert e_w <= 1.5 * e_p, (e_w, e_p)


def test_untrained_network_still_converges_to_tolerance(torch_cuda):
    """A randomly initialised network is a poor guess: the sweeps still reach
    tol, and the result is as accurate as the plain one."""
    from paper_2412_00031_amd.warmstart import UNet, WarmStart
    torch = torch_cuda
    wl, s, xi, eta, src, par = _setup(torch, 4, first=20)
    ws = WarmStart(UNet("cuda", seed=123), wl["grid"])
    init = ws.predict(s, xi, eta, src, par)
    assert torch.isfinite(init).all()
    tau_p, st_p = _solve(torch, wl, s, xi, eta, src, par, 1e-6)
    tau_w, st_w = _solve(torch, wl, s, xi, eta, src, par, 1e-6, init)
    tau_r, _ = _solve(torch, wl, s, xi, eta, src, par, 1e-13)
    assert (st_w.cpu().numpy() > 0).all()
    e_p = float((tau_p - tau_r).abs().max())
    e_w = float((tau_w - tau_r).abs().max())
    assert e_w <= 2.0 * e_p, (e_w, e_p)


def test_warm_start_on_finer_121_grid(torch_cuda):
    """The evaluation geometry (121^3, h = 0.83 km; the network was trained at
    h = 1 km): on 32 held-out sources the warm start still needs fewer
    iterations to tol 1e-6 and ends as close to the tol-1e-13 solution as the
    plain start."""
    from paper_2412_00031_amd.eval_warmstart import evaluate
    res = evaluate(nsrc=32, ref_sources=32, log=lambda m: None)
    print(res)
    assert res["warm"]["mean_iters"] < res["plain"]["mean_iters"]
    assert res["initial_error_mean"]["warm"] < 0.5 * res["initial_error_mean"]["plain"]
    fe = res["final_error_vs_tol_1e-13"]
    assert fe["warm_max"] <= 1.5 * fe["plain_max"], fe
