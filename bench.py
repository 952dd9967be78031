#!/usr/bin/env python3
"""Throughput of the adjoint-state traveltime hot path on one MI355X.

One step = one pass of the whole per-source path over a batch of sources:
source constants, (warm start: features, U-Net inference, interpolation to
the initial tau), forward fast-sweeping solve to tol, receiver traveltimes,
misfit and adjoint sources (Eqs. (2), (A2)), adjoint solve to tol, and the
kernels summed over sources (Eqs. (6)-(8)).  Workload: 101^3 spherical grid
(0-100 km depth, 4 x 4 degrees), Gaussian-random-field slowness (+-10 %) and
anisotropy (+-0.04), 128 sources, 500 surface receivers, tol 1e-6, FP64;
observed times come from a forward solve in an independent random model
(computed before timing).

The solves of a timed step are asynchronous: each enqueues its iteration
budget and nothing waits on the host; converged sources exit on the device.
The budgets are per source (its iteration count in a host-polled calibration
step of the same start, plus a margin); each source group of a solve iterates
the largest budget of its sources.  After the timed steps every source's status is checked:
a source that reached its budget unconverged voids the value (null, exit 3).
The plain path (tau = 1 start) and the warm-started path run the same steps
back to back; value = sources per second (fwd + adjoint + kernel per source)
of the warm-started path, with the plain path's figures in "plain", and, on a
few steps each, the plain path host-polled, with its iterations replayed from
captured graphs, and with the upwind adjoint of Eq. (5).

Prints one JSON line.  Extra objects: "roofline" (both sweep kernels, timed
live with HIP event pairs around the back-to-back launches of each
directional sweep on the library's stream; the dominant one is reported),
"cpu_baseline" (converged oracle solves on all host cores, and on one
thread) and "aux" (the kernels that run once per inversion step outside the
solves -- kernel density, multiple-grid projection and expansion,
common-receiver misfit, relocation -- each timed on seeded inputs of the
workload's shapes against its algorithmic bytes, with the oracle's time for
the same call beside it).
"""
import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "converged fwd+adjoint Eikonal solves/s (101³, tol 1e-6), plain vs warm-start"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsrc", type=int, default=128)
    ap.add_argument("--tile-k", type=int, default=0, help="tile depth for both solves (0: autotune)")
    ap.add_argument("--tile-k-fwd", type=int, default=0, help="forward tile depth (overrides --tile-k/autotune)")
    ap.add_argument("--tile-k-adj", type=int, default=0, help="adjoint tile depth (overrides --tile-k/autotune)")
    ap.add_argument("--no-autotune", action="store_true", help="use the library's default tile depths")
    ap.add_argument("--no-sweep-timing", action="store_true",
                    help="skip the per-launch sweep events (roofline then unmeasured)")
    ap.add_argument("--obs", choices=("true-model", "straight"), default="true-model",
                    help="observed times: a forward solve in the independent true model (default), or straight-line "
                         "times (no solve before the measured steps; for counter runs)")
    ap.add_argument("--max-iter", type=int, default=1000,
                    help="iteration cap of the host-polled calibration and comparison steps")
    ap.add_argument("--budget-margin", type=int, default=8,
                    help="iterations added to each source's count in the calibration step to give its budget in "
                         "the asynchronous solves")
    ap.add_argument("--uniform-budget", action="store_true",
                    help="one budget per solve (the largest calibrated count plus the margin) instead of "
                         "per-source budgets")
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="timed steps of the comparison paths (host-polled, graph replay, continuous adjoint); 0 "
                         "skips them")
    ap.add_argument("--cpu-baseline", choices=("full", "all-cores", "off"), default="full",
                    help="converged oracle solves on all host cores (and one thread with 'full')")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_const", const="off")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--cpu-sources", type=int, default=0,
                    help="oracle sources of the all-core run (default: one per thread)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB of a plain device-to-device copy run first (counter calibration)")
    ap.add_argument("--start", choices=("both", "plain", "warm"), default="both",
                    help="which forward start to time (both: plain, then warm-started)")
    ap.add_argument("--weights", default=None, help="U-Net weights (.npz) of the warm start")
    ap.add_argument("--groups", type=int, default=0,
                    help="concurrently iterated source groups of each solve (0: autotuned, or the library "
                         "default with --no-autotune)")
    ap.add_argument("--order", choices=("iterations", "natural"), default="iterations",
                    help="source order of the batch: by the iteration counts of a host-polled forward solve "
                         "before the timed region, most first, so that each source group holds sources that "
                         "converge together (iterations), or as generated (natural)")
    ap.add_argument("--tune-iters", action="store_true",
                    help="tune the source groups on a few iterations of the whole batch instead of whole "
                         "solves to tol")
    ap.add_argument("--adjoint", choices=("discrete", "continuous"), default="discrete",
                    help="adjoint of the timed steps: the exact discrete transpose (default) or the upwind "
                         "discretisation of Eq. (5)")
    ap.add_argument("--aux-only", action="store_true",
                    help="time only the per-step kernels outside the solves (kernel density, multiple-grid "
                         "projection/expansion, common-receiver misfit) and print their object")
    ap.add_argument("--no-aux", action="store_true", help="skip the auxiliary-kernel timings")
    ap.add_argument("--roofline-only", action="store_true",
                    help="run only the roofline step (sweep kernels timed per directional sweep)")
    return ap.parse_args()


SOLVER_SOURCES = ("tt_kernels.hip", "tt_device.h", "tt_internal.h")


def solver_sha256():
    """sha256 over the device sources the sweep kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    for name in SOLVER_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2412_00031_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, updates_per_launch, tile_k):
    """HBM bytes per launch of `kernel` at tile depth `tile_k` from the
    committed rocprofv3 counter summary (bytes per node update, calibrated
    against a plain copy, for each profiled tile depth), or None when the
    solver sources (SOLVER_SOURCES) changed since the counters were taken or
    that tile depth was not profiled."""
    path = os.path.join(ROOT, "profiles", "sweeps_sph101_pmc.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith(("|", "`", "#")):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sha256") != solver_sha256():
        return None
    try:
        per_update = (float(vals[f"{kernel} tile_k {tile_k} read_bytes_per_update"]) +
                      float(vals[f"{kernel} tile_k {tile_k} write_bytes_per_update"]))
    except KeyError:
        return None
    return per_update * updates_per_launch


def interior_nonfixed(grid):
    n = grid["n"]
    return (n[0] - 2) * (n[1] - 2) * (n[2] - 2)


def cpu_baseline(wl, nsrc, threads):
    """Converged oracle solves timed on host threads: `nsrc` sources of the
    workload, one per thread at a time (`threads` threads), each a forward
    solve to tol, its adjoint solve to tol at the workload's seeded adjoint
    sources and its kernel contribution.  Returns (solves/s, wall s, mean
    forward and adjoint iterations)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle as O
    g, s, xi, eta = wl["grid"], wl["s"], wl["xi"], wl["eta"]
    src = wl["src"][:nsrc]
    par = O.source_params(g, s, xi, eta, src)
    kappa, tol = wl["kappa"], wl["tol"]

    def solve(q):
        tau, itf, cf, _ = O.forward(g, s, xi, eta, src[q], par[q], kappa, tol, 1000)
        rhs = O.adjoint_rhs(g, src[q], par[q], wl["rec"], wl["R"][q])
        lam, ita, ca, _ = O.adjoint(g, s, xi, eta, src[q], par[q], kappa, tau, rhs, tol, 1000)
        O.kernel(g, s, xi, eta, src[q], par[q], kappa, tau, lam)
        if not (cf and ca):
            raise RuntimeError(f"oracle source {q} did not converge")
        return itf, ita

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        its = list(ex.map(solve, range(nsrc)))
    wall = time.perf_counter() - t0
    its = np.array(its, dtype=float)
    return nsrc / wall, wall, float(its[:, 0].mean()), float(its[:, 1].mean())


AUX_GRIDS = dict(m=(11, 13, 13), H=5)
AUX_CR_PER_REC = 64


def aux_inputs(wl, nsrc):
    """Seeded synthetic inputs for the per-step kernels outside the solves, with
    the workload's shapes: gradient fields [3, N] and an adjoint density field
    [N], H = 5 staggered 11 x 13 x 13 inversion grids, traveltimes [nsrc, nrec]
    and 64 common-receiver source pairs per receiver."""
    import numpy as np
    from paper_2412_00031_amd import workloads as W
    g = wl["grid"]
    n = tuple(g["n"])
    rng = np.random.default_rng(9001)
    grad = rng.standard_normal((3,) + n)
    dens = np.abs(rng.standard_normal(n)) + 0.1
    inv = W.staggered_inversion_grids(g, AUX_GRIDS["m"], AUX_GRIDS["H"])
    C = [rng.standard_normal((3,) + tuple(len(c) for c in axes)) for axes in inv]
    nrec = len(wl["rec"])
    T = rng.uniform(5.0, 30.0, (nsrc, nrec))
    T_obs = T + rng.normal(0.0, 0.2, T.shape)
    off, pair, tri = W.receiver_source_pairs(nsrc, nrec, AUX_CR_PER_REC, rng)
    wcr = rng.uniform(0.5, 2.0, len(tri))
    Rr = rng.normal(0.0, 0.1, (len(wl["src"]), nrec))
    return dict(grad=grad, dens=dens, inv=inv, C=C, T=T, T_obs=T_obs, off=off, pair=pair, tri=tri, wcr=wcr,
                eps=1e-3, zeta=0.5, gamma=1.0, Rr=Rr)


def aux_gpu(wl, a, dev, reps=20):
    """Average time of one call of each per-step entry point outside the solves
    (one or two kernel launches), by
    torch events on the stream the kernels run on (torch's current stream,
    which the binding passes to the library), and its algorithmic HBM bytes."""
    import ctypes
    import numpy as np
    import torch
    from paper_2412_00031_amd import _lib, api
    lib = _lib.load()
    g = wl["grid"]
    N = int(np.prod(g["n"]))
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    s, grad, dens = t(wl["s"]), t(a["grad"]), t(a["dens"])
    m, coords, sizes = api._mg_args(a["inv"], dev)
    M = sum(3 * x * y * z for x, y, z in sizes)
    proj = torch.empty(M, dtype=torch.float64, device=dev)
    nws = int(lib.tt_mg_workspace_size(ctypes.byref(api._grid(g)), len(sizes), m))
    mg_ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
    Cf = t(np.concatenate([c.reshape(-1) for c in a["C"]]))
    field = torch.empty((3, N), dtype=torch.float64, device=dev)
    gr = api._grid(g)
    T, Tobs = t(a["T"]), t(a["T_obs"])
    off, pair, wcr = t(a["off"], torch.int32), t(a["pair"], torch.int32), t(a["wcr"])
    R = torch.zeros_like(T)
    chi = torch.zeros((), dtype=torch.float64, device=dev)
    # relocation: receiver-side fields (tau = 1, i.e. Gamma_m = T0 of the receiver; the
    # kernels' cost does not depend on the values) sampled at the workload's sources
    recd, evd = t(wl["rec"]), t(wl["src"])
    nfield, nev = recd.shape[0], evd.shape[0]
    fpar = api.source_params(g, s, t(wl["xi"]), t(wl["eta"]), recd)
    ftau = torch.ones((nfield, N), dtype=torch.float64, device=dev)
    rws = api.workspace(g, nfield, 2, 0, dev)
    Rr = t(a["Rr"])
    cp = lambda x: ctypes.c_void_p(x.data_ptr())
    st = lambda: ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    calls = {
        "tt_kernel_density": (lambda: api.kernel_density(g, s, dens, grad, a["eps"], a["zeta"]), 72.0 * N, "hbm"),
        "tt_mg_project": (lambda: _lib.check(lib.tt_mg_project(ctypes.byref(gr), len(sizes), m, cp(coords), cp(grad),
                                                                cp(proj), cp(mg_ws), ctypes.c_size_t(nws), st())),
                         24.0 * N + 8.0 * M, "hbm"),
        "tt_mg_expand": (lambda: _lib.check(lib.tt_mg_expand(ctypes.byref(gr), len(sizes), m, cp(coords), cp(Cf),
                                                              cp(field), st())), 24.0 * N + 8.0 * M, "hbm"),
        "tt_misfit_cr": (lambda: api.misfit_cr(T, Tobs, off, pair, wcr, a["gamma"], R, chi),
                        80.0 * len(a["tri"]), "latency"),
        # algorithmic: the 8 corners of every (earthquake, field) pair, read once
        "tt_reloc_times": (lambda: api.reloc_times(g, recd, fpar, ftau, evd, ws=rws), 64.0 * nev * nfield + 8.0 * nev * nfield,
                           "latency"),
        "tt_reloc_kernel": (lambda: api.reloc_kernel(g, recd, fpar, ftau, evd, Rr, ws=rws),
                            64.0 * nev * nfield + 8.0 * nev * nfield, "latency"),
    }
    kernels = {"tt_kernel_density": "k_kernel_density", "tt_mg_project": "k_mg_proj_planes + k_mg_proj_final",
               "tt_mg_expand": "k_mg_expand_planes", "tt_misfit_cr": "k_misfit_cr_R + k_misfit_cr_chi",
               "tt_reloc_times": "k_reloc_times", "tt_reloc_kernel": "k_reloc_kernel"}
    out = {}
    for name, (fn, nbytes, bound) in calls.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"kernels": kernels[name], "avg_call_ms": round(ms, 4), "algorithmic_bytes": int(nbytes),
                     "achieved": round(gbs, 1), "unit": "GB/s", "bound": bound}
        if bound == "hbm":
            out[name].update(peak=HBM_PEAK_GBS, frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def aux_cpu(wl, a):
    """The oracle's version of each auxiliary kernel on the same inputs, one
    thread, one call each (part of the CPU baseline leg)."""
    import oracle as O
    g = wl["grid"]
    out = {}
    t0 = time.perf_counter()
    O.kernel_density(g, wl["s"], a["dens"], a["grad"], a["eps"], a["zeta"])
    out["tt_kernel_density"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.mg_project(g, a["inv"], a["grad"])
    out["tt_mg_project"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.mg_expand(g, a["inv"], a["C"])
    out["tt_mg_expand"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.misfit_cr(a["T"], a["T_obs"], a["tri"], a["wcr"], a["gamma"])
    out["tt_misfit_cr"] = time.perf_counter() - t0
    # relocation on 8 earthquakes x 50 fields, scaled to all of them
    import numpy as np
    nf = 50
    fpar = O.source_params(g, wl["s"], wl["xi"], wl["eta"], wl["rec"][:nf])
    ftau = np.ones((nf,) + tuple(g["n"]))
    ev = wl["src"][:8]
    scale = len(wl["src"]) / len(ev) * len(wl["rec"]) / nf
    t0 = time.perf_counter()
    O.reloc_times(g, wl["rec"][:nf], fpar, ftau, ev)
    out["tt_reloc_times"] = (time.perf_counter() - t0) * scale
    t0 = time.perf_counter()
    O.reloc_kernel(g, wl["rec"][:nf], fpar, ftau, ev, a["Rr"][:8, :nf])
    out["tt_reloc_kernel"] = (time.perf_counter() - t0) * scale
    del ftau
    return {k: round(v * 1e3, 3) for k, v in out.items()}


def aux_section(wl, nsrc, dev, with_cpu):
    a = aux_inputs(wl, nsrc)
    res = aux_gpu(wl, a, dev)
    if with_cpu:
        for k, ms in aux_cpu(wl, a).items():
            res[k]["oracle_ms"] = ms
            res[k]["oracle_cores"] = 1
    res["inputs"] = (f"101^3 grid; {AUX_GRIDS['H']} staggered {AUX_GRIDS['m']} inversion grids; {nsrc} sources x "
                     f"{len(wl['rec'])} receivers with {AUX_CR_PER_REC} source pairs per receiver; relocation of the "
                     f"{len(wl['src'])} sources as earthquakes against {len(wl['rec'])} receiver-side fields; seeded "
                     f"synthetic fields; average of 20 calls after 3 (oracle: one call, relocation on 8 earthquakes "
                     f"scaled)")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the sources of a batch shard "
              "across GPUs with no communication, and this benchmark measures one GPU's share", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2412_00031_amd import _lib, api, workloads as W

    dev = torch.device("cuda:0")
    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 8
        xa = torch.ones(n, dtype=torch.float64, device=dev)
        xb = torch.empty_like(xa)
        torch.cuda.synchronize()
        xb.copy_(xa)
        torch.cuda.synchronize()
        del xa, xb
        log(f"copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written")
    wl = W.sph101(nsrc=args.nsrc)
    g, kappa, tol = wl["grid"], wl["kappa"], wl["tol"]
    if args.aux_only:
        print(json.dumps({"aux": aux_section(wl, args.nsrc, dev, args.cpu_baseline != "off")}), flush=True)
        return
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    s, xi, eta, src, rec = t(wl["s"]), t(wl["xi"]), t(wl["eta"]), t(wl["src"]), t(wl["rec"])
    nsrc = args.nsrc
    lib = _lib.load()

    if args.obs == "true-model":
        # observations: forward solve in the independent "true" model (untimed)
        st_, xt_, et_ = t(wl["s_true"]), t(wl["xi_true"]), t(wl["eta_true"])
        par_t = api.source_params(g, st_, xt_, et_, src)
        tau_t, st_t = api.forward(g, st_, xt_, et_, src, par_t, tol, 1000, kappa, poll=True)
        T_obs = api.sample(g, src, par_t, tau_t, rec)
        del tau_t
        torch.cuda.synchronize()
        if (st_t <= 0).any():
            sys.exit("observations: the true-model forward solve did not converge")
    else:
        T_obs = t(W.straight_line_times(g, wl["src"], wl["rec"], 6.4))
    log(f"observations ready ({args.obs})")

    if args.order == "iterations" and not args.roofline_only:
        # scheduling input, like the tuner's choices: sources that take the
        # most iterations first, so that each contiguous source group holds
        # sources that converge together and a group's launches do not carry
        # one slow source through a tail of otherwise finished ones (the
        # roofline step runs one group, where the order does not matter)
        par0 = api.source_params(g, s, xi, eta, src)
        _, st0 = api.forward(g, s, xi, eta, src, par0, tol, 1000, kappa, poll=True)
        c0 = st0.cpu().numpy()
        if (c0 <= 0).any():
            sys.exit("ordering: the forward solve did not converge")
        perm = torch.as_tensor(np.argsort(-c0, kind="stable"), device=dev)
        src, T_obs = src[perm].contiguous(), T_obs[perm].contiguous()
        del par0, st0
        log(f"sources ordered by forward iterations ({int(c0.max())} .. {int(c0.min())})")

    tk_f = args.tile_k_fwd or args.tile_k
    tk_a = args.tile_k_adj or args.tile_k
    gr_f = gr_a = args.groups
    tuned = None
    if (tk_f == 0 or tk_a == 0) and not args.no_autotune:
        from paper_2412_00031_amd import autotune
        par0 = api.source_params(g, s, xi, eta, src)
        tuned = autotune.tune(g, s, xi, eta, src, par0, kappa, rec, log=log,
                              tol=None if args.tune_iters else tol)
        tk_f, tk_a = tk_f or tuned["fwd"], tk_a or tuned["adj"]
        if args.groups == 0:
            gr_f, gr_a = tuned["groups_fwd"], tuned["groups_adj"]
    tk_f = tk_f or int(lib.tt_default_tile_k(0))
    tk_a = tk_a or int(lib.tt_default_tile_k(1))
    auto_groups = max(1, min(4, nsrc // 32))
    gr_f, gr_a = gr_f or auto_groups, gr_a or auto_groups
    log(f"tile depths: forward {tk_f}, adjoint {tk_a}; source groups: forward {gr_f}, adjoint {gr_a}")
    ws_f = api.workspace(g, nsrc, 0, tk_f, dev, groups=gr_f)
    ws_a = api.workspace(g, nsrc, 1, tk_a, dev, groups=gr_a)
    tau = torch.empty((nsrc,) + tuple(g["n"]), dtype=torch.float64, device=dev)
    lam = torch.empty_like(tau)
    grad = torch.empty((3,) + tuple(g["n"]), dtype=torch.float64, device=dev)
    st_f = torch.empty(nsrc, dtype=torch.int32, device=dev)
    st_a = torch.empty_like(st_f)

    warm = None
    if args.start != "plain":
        from paper_2412_00031_amd.warmstart import WEIGHTS, UNet, WarmStart
        wpath = args.weights or WEIGHTS
        if os.path.exists(wpath):
            warm = WarmStart(UNet.load(wpath, dev), g)
            init_buf = torch.empty((nsrc, tau[0].numel()), dtype=torch.float64, device=dev)
            log(f"warm start: {wpath}")
        elif args.start == "warm":
            sys.exit(f"no warm-start weights at {wpath}")
        else:
            log(f"no warm-start weights at {wpath}: timing the plain path only")

    budget = {"fwd": args.max_iter, "adj": args.max_iter, "fwd_src": None, "adj_src": None}

    def step(use_warm, poll=False, timed=False, graph=False, continuous=args.adjoint == "continuous"):
        par = api.source_params(g, s, xi, eta, src)
        init = warm.predict(s, xi, eta, src, par, out=init_buf) if use_warm else None
        api.forward(g, s, xi, eta, src, par, tol, budget["fwd"], kappa, tau_init=init, tile_k=tk_f, ws=ws_f,
                    out=tau, time_sweeps=timed, graph=graph, groups=gr_f, poll=poll, status=st_f,
                    budgets=budget["fwd_src"])
        T = api.sample(g, src, par, tau, rec)
        chi, R = api.misfit(T, T_obs)
        api.adjoint(g, s, xi, eta, src, par, tau, rec, R, tol, budget["adj"], kappa, tile_k=tk_a, ws=ws_a, out=lam,
                    time_sweeps=timed, graph=graph, groups=gr_a, continuous=continuous, poll=poll, status=st_a,
                    budgets=budget["adj_src"])
        api.kernel(g, s, xi, eta, src, par, tau, lam, grad=grad.zero_())
        return chi

    def run(name, steps, warmup, fn):
        for w in range(warmup):
            fn()
            torch.cuda.synchronize()
        log(f"{name}: {warmup} warmup step(s) done")
        api.sweep_timing(0, reset=True)
        api.sweep_timing(1, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            chi = fn()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        f, a = st_f.cpu().numpy(), st_a.cpu().numpy()
        conv = bool((f > 0).all() and (a > 0).all())
        log(f"{name}: timed {steps} steps: {elapsed:.2f} s ({1e3 * elapsed / steps:.1f} ms per step)"
            + ("" if conv else f"; NOT CONVERGED (fwd {f.min()}, adj {a.min()})"))
        return dict(elapsed=elapsed, steps=steps, it_f=np.abs(f), it_a=np.abs(a), chi=float(chi), converged=conv,
                    sweep=(api.sweep_timing(0, reset=True), api.sweep_timing(1, reset=True)))

    # Iteration budgets of the asynchronous solves: a host-polled step of each
    # start finds every source's iteration counts, and its budget is its count
    # plus a margin (each source group iterates the largest budget of its
    # sources); every timed step's statuses are checked afterwards.
    def calibrate(use_warm, continuous=False):
        step(use_warm, poll=True, continuous=continuous)
        torch.cuda.synchronize()
        f, a = st_f.cpu().numpy(), st_a.cpu().numpy()
        if (f <= 0).any() or (a <= 0).any():
            sys.exit(f"calibration step did not converge within {args.max_iter} iterations")
        return f.astype(np.int32), a.astype(np.int32)

    def with_budget(fc, ac, fn):
        fb, ab = fc + args.budget_margin, ac + args.budget_margin
        def wrapped():
            budget["fwd"], budget["adj"] = int(fb.max()), int(ab.max())
            budget["fwd_src"], budget["adj_src"] = (None, None) if args.uniform_budget else (fb, ab)
            try:
                return fn()
            finally:  # the other steps (host-polled) run to convergence within max_iter
                budget.update(fwd=args.max_iter, adj=args.max_iter, fwd_src=None, adj_src=None)
        return wrapped

    runs, budgets, cal = {}, {}, {}
    if not args.roofline_only:
        cal["plain"] = calibrate(False)
        if warm is not None:
            cal["warm"] = calibrate(True)
        budgets = {k: {"fwd": [int(v[0].min()) + args.budget_margin, int(v[0].max()) + args.budget_margin],
                       "adj": [int(v[1].min()) + args.budget_margin, int(v[1].max()) + args.budget_margin]}
                   for k, v in cal.items()}
        log(f"iteration budgets (polled count + {args.budget_margin}, "
            f"{'largest per solve' if args.uniform_budget else 'per source'}; min, max): {budgets}")
    if not args.roofline_only:
        runs["plain"] = run("plain", args.steps, args.warmup, with_budget(*cal["plain"], lambda: step(False)))
        if warm is not None:
            runs["warm"] = run("warm", args.steps, args.warmup, with_budget(*cal["warm"], lambda: step(True)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                warm.predict(s, xi, eta, src, api.source_params(g, s, xi, eta, src), out=init_buf)
            torch.cuda.synchronize()
            runs["warm"]["predict_ms"] = (time.perf_counter() - t0) / 3 * 1e3
        if args.compare_steps > 0:
            cs = args.compare_steps
            # the same plain step host-polled, and with iterations replayed from captured graphs
            runs["plain_polled"] = run("plain, host-polled", cs, 1, lambda: step(False, poll=True))
            runs["plain_graph"] = run("plain, graph replay", cs, 1,
                                      with_budget(*cal["plain"], lambda: step(False, graph=True)))
            if args.adjoint == "discrete":
                # the plain-start step with the upwind adjoint of Eq. (5) (the paper's route)
                runs["continuous"] = run("plain, continuous adjoint", cs, 1,
                                         lambda: step(False, poll=True, continuous=True))
    # roofline step: the same step once more with every directional sweep of the
    # sweep kernels timed by HIP events on the library's stream (one source
    # group, so each launch carries a tile-plane of every active source)
    rf = None
    if not args.no_sweep_timing:
        rf = run("roofline step", 1, 0 if runs else args.warmup,
                 lambda: step(warm is not None, poll=True, timed=True))
    main_run = rf if args.roofline_only else (runs["warm"] if warm is not None else runs["plain"])
    elapsed, it_f, it_a = main_run["elapsed"], main_run["it_f"], main_run["it_a"]
    steps_main = main_run["steps"]
    all_converged = all(r["converged"] for r in list(runs.values()) + ([rf] if rf else []))

    value = nsrc * steps_main / elapsed
    roofline = None
    if rf is not None:
        (ms_f, n_f), (ms_a, n_a) = rf["sweep"]
        nodes = interior_nonfixed(g) - 8
        # algorithmic bytes per node update: forward = tau read + write (16 B)
        # plus the model's s, xi, eta (24 B per node per sweep, shared by the
        # batch); adjoint = lambda read + write (16 B) plus 32 B of stored
        # coefficients plus the shared model (the right-hand side, read only
        # in the tiles at the receivers, is not counted)
        upd_f = float(rf["it_f"].sum()) * 8 * nodes
        upd_a = float(rf["it_a"].sum()) * 8 * nodes
        bytes_f = upd_f * (16.0 + 24.0 / nsrc)
        bytes_a = upd_a * (16.0 + 32.0 + 24.0 / nsrc)
        kern = {
            "k_fwd_sweep": dict(ms=ms_f, launches=n_f, bytes=bytes_f, updates=upd_f, tk=tk_f),
            "k_adj_sweep": dict(ms=ms_a, launches=n_a, bytes=bytes_a, updates=upd_a, tk=tk_a),
        }
        for K in kern.values():
            K["achieved"] = K["bytes"] / (K["ms"] * 1e-3) / 1e9 if K["ms"] > 0 else 0.0
        dom = max(kern, key=lambda k: kern[k]["ms"])
        K = kern[dom]
        avg_ms = K["ms"] / max(K["launches"], 1)
        traffic = measured_traffic(dom, K["updates"] / max(K["launches"], 1), K["tk"])
        roofline = {
            "bound": "hbm", "achieved": round(K["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(K["achieved"] / HBM_PEAK_GBS, 4), "traffic": None if traffic is None else round(traffic),
            "algorithmic_bytes_per_launch": round(K["bytes"] / max(K["launches"], 1)),
            "kernel": dom, "avg_launch_ms": round(avg_ms, 5), "launches": K["launches"],
            "bytes_per_update": round(K["bytes"] / K["updates"], 3),
            "sweep_ms": {k: round(v["ms"], 2) for k, v in kern.items()},
            "frac_by_kernel": {k: round(v["achieved"] / HBM_PEAK_GBS, 4) for k, v in kern.items()},
            "region": "one extra step after the timed ones, host-polled, one source group, every directional sweep "
                      "timed",
        }

    cpu = None
    if args.cpu_baseline != "off":
        cores = len(os.sched_getaffinity(0))
        threads = args.cpu_threads or cores
        n_all = min(nsrc, max(threads, args.cpu_sources))
        log(f"cpu baseline: {n_all} converged oracle solves on {threads} threads")
        v_all, wall, mf, ma = cpu_baseline(wl, n_all, threads)
        cpu = {"value": round(v_all, 5), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"{n_all} sources of the workload, each solved by the oracle to convergence (forward and "
                         f"adjoint to tol {tol:g}, mean {mf:.1f} / {ma:.1f} iterations, at the workload's seeded "
                         f"adjoint sources) and its kernel accumulated, {threads} host threads "
                         f"(sched_getaffinity: {cores} cores), {wall:.1f} s wall"}
        if args.cpu_baseline == "full":
            v1, wall1, mf1, ma1 = cpu_baseline(wl, 1, 1)
            cpu["one_thread"] = {"value": round(v1, 5), "unit": "solves/s", "cores": 1,
                                 "sample": f"source 0 converged on one thread ({wall1:.1f} s)"}
        log(f"cpu baseline: {cpu['value']} solves/s")

    aux = None
    if not args.no_aux:
        log("auxiliary kernels")
        aux = aux_section(wl, nsrc, dev, args.cpu_baseline != "off")

    def summary(r):
        return {"value": round(nsrc * r["steps"] / r["elapsed"], 4), "ms_per_step": round(1e3 * r["elapsed"] / r["steps"], 2),
                "steps": r["steps"], "mean_iters_fwd": round(float(r["it_f"].mean()), 2),
                "mean_iters_adj": round(float(r["it_a"].mean()), 2), "chi": r["chi"], "converged": r["converged"]}

    start = "warm start (U-Net prediction, plain sweeps to the same tol)" if warm is not None else "plain start"
    line = {
        "metric": METRIC, "value": round(value, 4) if all_converged else None, "unit": "solves/s", "n_gpus": 1,
        "steps": steps_main, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / steps_main, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "plain": summary(runs["plain"]) if "plain" in runs else None,
        "warm": dict(summary(runs["warm"]), predict_ms=round(runs["warm"]["predict_ms"], 2)) if "warm" in runs else None,
        "plain_host_polled": summary(runs["plain_polled"]) if "plain_polled" in runs else None,
        "plain_graph_replay": summary(runs["plain_graph"]) if "plain_graph" in runs else None,
        "plain_continuous_adjoint": summary(runs["continuous"]) if "continuous" in runs else None,
        "roofline_only": bool(args.roofline_only),
        "config": {"workload": f"sph101: 101^3 spherical (0-100 km, 4x4 deg), GRF model, {nsrc} sources, "
                               f"{len(wl['rec'])} receivers, tol {tol:g}, {start}",
                   "nsrc": nsrc, "grid": list(g["n"]), "tol": tol, "kappa": kappa,
                   "mean_iters_fwd": round(float(it_f.mean()), 2), "mean_iters_adj": round(float(it_a.mean()), 2),
                   "tile_k": {"fwd": tk_f, "adj": tk_a,
                              "chosen_by": "autotune" if tuned else ("fixed" if (args.tile_k_fwd or args.tile_k_adj
                                                                                 or args.tile_k) else "default")},
                   "source_groups": {"fwd": gr_f, "adj": gr_a},
                   "source_order": ("by forward iterations of a host-polled solve before timing, most first"
                                    if args.order == "iterations" else "as generated"),
                   "solves": "asynchronous (iteration budget, no host polling)", "iteration_budgets": budgets,
                   "budget_rule": (f"largest calibrated count + {args.budget_margin} per solve" if args.uniform_budget
                                   else f"calibrated count + {args.budget_margin} per source, the largest of a "
                                        "source group's budgets for the group"),
                   "adjoint": args.adjoint},
        "roofline": roofline, "cpu_baseline": cpu, "aux": aux,
    }
    if not all_converged:
        line["error"] = "not every source converged within its iteration budget"
    print(json.dumps(line), flush=True)
    if not all_converged and not args.roofline_only:
        sys.exit(3)


if __name__ == "__main__":
    main()
