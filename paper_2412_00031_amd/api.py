"""Python binding of libtt: argument marshalling over torch device tensors.

Every function here hands device pointers to the C ABI (include/tt.h) and
returns torch tensors; no step of the computation happens in Python.  PyTorch
provides device memory and the current stream only.

Grid description: a mapping with ``n`` (3 ints), ``coord`` (0 Cartesian
z/y/x km, 1 spherical r km / latitude rad / longitude rad), ``o`` and ``h``.
"""
import ctypes

import numpy as np
import torch

from . import _lib

_F64 = torch.float64


def _grid(grid):
    g = _lib.TTGrid()
    for a in range(3):
        g.n[a] = int(grid["n"][a])
        g.o[a] = float(grid["o"][a])
        g.h[a] = float(grid["h"][a])
    g.coord = int(grid["coord"])
    return g


def _budgets(budgets, nsrc):
    """Host int32 copy of per-source iteration budgets (kept alive by the
    caller for the duration of the call), or None."""
    if budgets is None:
        return None
    b = np.ascontiguousarray(np.asarray(budgets.cpu() if isinstance(budgets, torch.Tensor) else budgets,
                                        dtype=np.int32).reshape(-1))
    if b.size != nsrc:
        raise ValueError(f"budgets must have one entry per source ({nsrc}), got {b.size}")
    return b


def _opts(tol, max_iter, kappa, tile_k=0, time_sweeps=False, eps_hist=None, graph=False, groups=0, continuous=False,
          poll=False, compact=False, budgets=None, adjoint_init=False):
    o = _lib.TTOpts()
    o.budgets = budgets.ctypes.data if budgets is not None else None
    o.groups = int(groups)
    o.eps_hist = _dev(eps_hist, "eps_hist").value if eps_hist is not None else None
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.kappa = float(kappa)
    o.tile_k = int(tile_k)
    o.flags = ((_lib.TT_FLAG_TIME_SWEEPS if time_sweeps else 0) | (_lib.TT_FLAG_GRAPH if graph else 0)
               | (_lib.TT_FLAG_CONTINUOUS_ADJOINT if continuous else 0) | (_lib.TT_FLAG_POLL if poll else 0)
               | (_lib.TT_FLAG_COMPACT_ADJOINT if compact else 0) | (_lib.TT_FLAG_ADJOINT_INIT if adjoint_init else 0))
    return o


def sweep_timing(which, reset=True):
    """(total ms, launches) of the timed sweep-kernel launches of this thread:
    which = 0 forward, 1 adjoint (calls made with time_sweeps=True)."""
    lib = _lib.load()
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _lib.check(lib.tt_sweep_timing(int(which), ctypes.byref(ms), ctypes.byref(n), int(bool(reset))))
    return ms.value, n.value


def _dev(t, name, dtype=_F64, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a GPU device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _null():
    return ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _N(grid):
    n = grid["n"]
    return int(n[0]) * int(n[1]) * int(n[2])


def workspace(grid, nsrc, which, tile_k=0, device=None, groups=0, time_sweeps=False, compact=False):
    """Device workspace (uint8 tensor) for forward (0), adjoint (1), sample (2), kernel (3);
    groups / time_sweeps / compact as for the solve that will use it (its size
    depends on the number of source groups and, for the adjoint, on the record
    layout).  An empty batch needs no workspace: zero bytes."""
    lib = _lib.load()
    if int(nsrc) == 0:
        return torch.empty(0, dtype=torch.uint8, device=device)
    g = _grid(grid)
    o = _opts(1e-6, 1, 1.0, tile_k, time_sweeps=time_sweeps, groups=groups, compact=compact)
    nbytes = lib.tt_workspace_size(ctypes.byref(g), int(nsrc), ctypes.byref(o), int(which))
    if nbytes == 0:
        raise ValueError("invalid grid or source count for the workspace")
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def source_params(grid, s, xi, eta, src_pos):
    """s0, xi0, eta0 at each source (trilinear interpolation of the model)."""
    lib = _lib.load()
    N = _N(grid)
    nsrc = src_pos.shape[0]
    par = torch.empty((nsrc, 3), dtype=_F64, device=s.device)
    g = _grid(grid)
    _lib.check(lib.tt_source_params(ctypes.byref(g), _dev(s, "s", numel=N), _dev(xi, "xi", numel=N),
                                    _dev(eta, "eta", numel=N), int(nsrc), _dev(src_pos, "src_pos", numel=3 * nsrc),
                                    _dev(par, "src_par"), _stream(s.device)))
    return par


def forward(grid, s, xi, eta, src_pos, src_par, tol, max_iter, kappa, tau_init=None, tile_k=0, ws=None,
            out=None, time_sweeps=False, eps_hist=None, graph=False, groups=0, poll=False, status=None,
            budgets=None):
    """Batched forward solve.  Returns (tau [nsrc, *n], status int32 [nsrc]).
    eps_hist: optional float64 device tensor [nsrc, max_iter] receiving the
    convergence measure of every iteration.  groups: concurrently iterated
    source groups (0 = library default; results do not depend on it).
    poll=False (the library's default) enqueues exactly max_iter iterations on
    the current stream and returns at once (capturable; max_iter is the
    iteration budget and status is written on the device); poll=True stops as
    soon as every source has converged and returns after completion.
    budgets: optional per-source iteration budgets (host sequence of nsrc ints
    in [1, max_iter]); each source group iterates the largest of its own."""
    lib = _lib.load()
    N = _N(grid)
    nsrc = int(src_pos.shape[0])
    dev = s.device
    tau = out if out is not None else torch.empty((nsrc,) + tuple(int(v) for v in grid["n"]), dtype=_F64, device=dev)
    if status is None:
        status = torch.empty(nsrc, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(grid, nsrc, 0, tile_k, dev, groups, time_sweeps)
    g = _grid(grid)
    if eps_hist is not None and eps_hist.numel() != nsrc * int(max_iter):
        raise ValueError("eps_hist must have nsrc * max_iter elements")
    bud = _budgets(budgets, nsrc)
    o = _opts(tol, max_iter, kappa, tile_k, time_sweeps, eps_hist, graph, groups, poll=poll, budgets=bud)
    ti = _dev(tau_init, "tau_init", numel=nsrc * N) if tau_init is not None else _null()
    _lib.check(lib.tt_forward(ctypes.byref(g), _dev(s, "s", numel=N), _dev(xi, "xi", numel=N),
                              _dev(eta, "eta", numel=N), nsrc, _dev(src_pos, "src_pos", numel=3 * nsrc),
                              _dev(src_par, "src_par", numel=3 * nsrc), ti, ctypes.byref(o),
                              _dev(tau, "tau", numel=nsrc * N), _dev(status, "status", torch.int32),
                              _dev(ws, "ws", torch.uint8), ws.numel(), _stream(dev)))
    return tau, status


def forward_noalloc(grid, s, xi, eta, src_pos, src_par, tol, max_iter, kappa, tau, status, tau_init=None, tile_k=0,
                    eps_hist=None):
    """tt_forward_noalloc: the asynchronous forward solve on the library's own
    fixed device scratch (no workspace, no allocation by the library).  The
    caller passes the outputs tau [nsrc, *n] and status int32 [nsrc]; one
    source group on the current stream; calls on one device must not overlap."""
    lib = _lib.load()
    N = _N(grid)
    nsrc = int(src_pos.shape[0])
    g = _grid(grid)
    o = _opts(tol, max_iter, kappa, tile_k, False, eps_hist)
    ti = _dev(tau_init, "tau_init", numel=nsrc * N) if tau_init is not None else _null()
    _lib.check(lib.tt_forward_noalloc(ctypes.byref(g), _dev(s, "s", numel=N), _dev(xi, "xi", numel=N),
                                      _dev(eta, "eta", numel=N), nsrc, _dev(src_pos, "src_pos", numel=3 * nsrc),
                                      _dev(src_par, "src_par", numel=3 * nsrc), ti, ctypes.byref(o),
                                      _dev(tau, "tau", numel=nsrc * N), _dev(status, "status", torch.int32,
                                                                               numel=nsrc), _stream(s.device)))
    return tau, status


def sample(grid, src_pos, src_par, tau, rec_pos, ws=None):
    """Traveltimes [nsrc, nrec] at the receivers."""
    lib = _lib.load()
    N = _N(grid)
    nsrc, nrec = int(src_pos.shape[0]), int(rec_pos.shape[0])
    dev = tau.device
    out = torch.empty((nsrc, nrec), dtype=_F64, device=dev)
    if ws is None:
        ws = workspace(grid, nsrc, 2, 0, dev)
    g = _grid(grid)
    _lib.check(lib.tt_sample(ctypes.byref(g), nsrc, _dev(src_pos, "src_pos", numel=3 * nsrc),
                             _dev(src_par, "src_par", numel=3 * nsrc), _dev(tau, "tau", numel=nsrc * N), nrec,
                             _dev(rec_pos, "rec_pos", numel=3 * nrec), _dev(out, "T_rec"),
                             _dev(ws, "ws", torch.uint8), ws.numel(), _stream(dev)))
    return out


def reloc_times(grid, field_pos, field_par, tau, ev_pos, ev_t0=None, ws=None):
    """T [nev, nfield] = Gamma_m(x_n) + t_n (Eq. (10), App. B): field m is the
    forward solution with receiver m as the source (tau [nfield, *n])."""
    lib = _lib.load()
    nfield, nev = int(field_pos.shape[0]), int(ev_pos.shape[0])
    dev = tau.device
    T = torch.empty((nev, nfield), dtype=_F64, device=dev)
    if ws is None:
        ws = workspace(grid, max(nfield, 1), 2, 0, dev)
    g = _grid(grid)
    _lib.check(lib.tt_reloc_times(ctypes.byref(g), nfield, _dev(field_pos, "field_pos", numel=3 * nfield),
                                  _dev(field_par, "field_par", numel=3 * nfield),
                                  _dev(tau, "tau", numel=nfield * _N(grid)), nev,
                                  _dev(ev_pos, "ev_pos", numel=3 * nev),
                                  _dev(ev_t0, "ev_t0", numel=nev) if ev_t0 is not None else _null(), _dev(T, "T"),
                                  _dev(ws, "ws", torch.uint8), ws.numel(), _stream(dev)))
    return T


def reloc_kernel(grid, field_pos, field_par, tau, ev_pos, R, ws=None):
    """Eq. (10): K [nev, 4] = location kernel in grid coordinates (3) and the
    origin-time kernel, from R = d chi / d T [nev, nfield]."""
    lib = _lib.load()
    nfield, nev = int(field_pos.shape[0]), int(ev_pos.shape[0])
    dev = tau.device
    K = torch.empty((nev, 4), dtype=_F64, device=dev)
    if ws is None:
        ws = workspace(grid, max(nfield, 1), 2, 0, dev)
    g = _grid(grid)
    _lib.check(lib.tt_reloc_kernel(ctypes.byref(g), nfield, _dev(field_pos, "field_pos", numel=3 * nfield),
                                   _dev(field_par, "field_par", numel=3 * nfield),
                                   _dev(tau, "tau", numel=nfield * _N(grid)), nev,
                                   _dev(ev_pos, "ev_pos", numel=3 * nev), _dev(R, "R", numel=nev * nfield),
                                   _dev(K, "K"), _dev(ws, "ws", torch.uint8), ws.numel(), _stream(dev)))
    return K


def misfit(T_rec, T_obs, w=None, pairs=None, wpair=None, alpha=1.0, beta=1.0, cr=None, wcr=None, gamma=1.0):
    """chi = alpha chi_t + beta chi_cs [+ gamma chi_cr] (Eq. (1)) as a device
    scalar tensor, and adjoint sources R [nsrc, nrec].  cr = (cr_off [nrec+1],
    cr_pair [npair_cr, 2]) int32 device tensors: the source pairs of each
    receiver (see misfit_cr); wcr [npair_cr] or None."""
    lib = _lib.load()
    nsrc, nrec = int(T_rec.shape[0]), int(T_rec.shape[1])
    dev = T_rec.device
    R = torch.empty_like(T_rec)
    chi = torch.empty((), dtype=_F64, device=dev)
    npair = 0 if pairs is None else int(pairs.shape[0])
    _lib.check(lib.tt_misfit(nsrc, nrec, _dev(T_rec, "T_rec"), _dev(T_obs, "T_obs", numel=nsrc * nrec),
                             _dev(w, "w", numel=nsrc * nrec) if w is not None else _null(), npair,
                             _dev(pairs, "pairs", torch.int32, numel=2 * npair) if npair else _null(),
                             _dev(wpair, "wpair", numel=nsrc * npair) if wpair is not None else _null(),
                             float(alpha), float(beta), _dev(R, "R"), _dev(chi, "chi"), _stream(dev)))
    if cr is not None:
        misfit_cr(T_rec, T_obs, cr[0], cr[1], wcr, gamma, R, chi)
    return chi, R


def misfit_cr(T_rec, T_obs, cr_off, cr_pair, wcr, gamma, R, chi):
    """Adds gamma chi_cr (Eq. (4)) to chi and its adjoint sources (Eq. (A4)) to
    R, in place.  cr_off [nrec+1] int32: the source pairs recorded at receiver m
    are rows cr_off[m]..cr_off[m+1]-1 of cr_pair [npair_cr, 2] int32, each
    unordered pair at a receiver listed once; wcr [npair_cr] or None (= 1)."""
    lib = _lib.load()
    nsrc, nrec = int(T_rec.shape[0]), int(T_rec.shape[1])
    npc = int(cr_pair.shape[0])
    _lib.check(lib.tt_misfit_cr(nsrc, nrec, _dev(T_rec, "T_rec"), _dev(T_obs, "T_obs", numel=nsrc * nrec),
                                _dev(cr_off, "cr_off", torch.int32, numel=nrec + 1),
                                _dev(cr_pair, "cr_pair", torch.int32, numel=2 * npc) if npc else _null(),
                                _dev(wcr, "wcr", numel=npc) if wcr is not None else _null(), float(gamma),
                                _dev(R, "R", numel=nsrc * nrec), _dev(chi, "chi", numel=1), _stream(T_rec.device)))
    return chi, R


def adjoint(grid, s, xi, eta, src_pos, src_par, tau, rec_pos, R, tol, max_iter, kappa, tile_k=0, ws=None,
            out=None, time_sweeps=False, eps_hist=None, graph=False, groups=0, continuous=False, poll=False,
            status=None, compact=False, budgets=None, lam_init=None):
    """Batched adjoint solve.  Returns (lambda [nsrc, *n], status int32 [nsrc]);
    eps_hist, groups, poll and budgets as for forward.  continuous=True solves Eq. (5)
    by upwind finite volumes and returns P s V in place of lambda.
    compact=True keeps one node-order copy of the coefficient records (a
    ninth of the workspace at 101^3; slower sweeps, identical results).
    lam_init [nsrc, *n]: the iteration's initial field instead of 0 (e.g. the
    continuous adjoint's P s V); it may be the out tensor itself."""
    lib = _lib.load()
    N = _N(grid)
    nsrc, nrec = int(src_pos.shape[0]), int(rec_pos.shape[0])
    dev = s.device
    lam = out if out is not None else torch.empty((nsrc,) + tuple(int(v) for v in grid["n"]), dtype=_F64, device=dev)
    if lam_init is not None and lam_init.data_ptr() != lam.data_ptr():
        lam.copy_(lam_init.reshape(lam.shape))
    if status is None:
        status = torch.empty(nsrc, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(grid, nsrc, 1, tile_k, dev, groups, time_sweeps, compact)
    g = _grid(grid)
    if eps_hist is not None and eps_hist.numel() != nsrc * int(max_iter):
        raise ValueError("eps_hist must have nsrc * max_iter elements")
    bud = _budgets(budgets, nsrc)
    o = _opts(tol, max_iter, kappa, tile_k, time_sweeps, eps_hist, graph, groups, continuous, poll, compact,
              budgets=bud, adjoint_init=lam_init is not None)
    _lib.check(lib.tt_adjoint(ctypes.byref(g), _dev(s, "s", numel=N), _dev(xi, "xi", numel=N),
                              _dev(eta, "eta", numel=N), nsrc, _dev(src_pos, "src_pos", numel=3 * nsrc),
                              _dev(src_par, "src_par", numel=3 * nsrc), _dev(tau, "tau", numel=nsrc * N), nrec,
                              _dev(rec_pos, "rec_pos", numel=3 * nrec), _dev(R, "R", numel=nsrc * nrec),
                              ctypes.byref(o), _dev(lam, "lam", numel=nsrc * N), _dev(status, "status", torch.int32),
                              _dev(ws, "ws", torch.uint8), ws.numel(), _stream(dev)))
    return lam, status


def kernel(grid, s, xi, eta, src_pos, src_par, tau, lam, grad=None, ws=None):
    """Discrete gradients [3, *n] summed over sources; adds to grad if given."""
    lib = _lib.load()
    N = _N(grid)
    nsrc = int(src_pos.shape[0])
    dev = s.device
    acc = grad is not None
    if grad is None:
        grad = torch.empty((3,) + tuple(int(v) for v in grid["n"]), dtype=_F64, device=dev)
    if ws is None:
        ws = workspace(grid, max(nsrc, 1), 3, 0, dev)
    g = _grid(grid)
    _lib.check(lib.tt_kernel(ctypes.byref(g), _dev(s, "s", numel=N), _dev(xi, "xi", numel=N),
                             _dev(eta, "eta", numel=N), nsrc, _dev(src_pos, "src_pos", numel=3 * nsrc),
                             _dev(src_par, "src_par", numel=3 * nsrc), _dev(tau, "tau", numel=nsrc * N),
                             _dev(lam, "lam", numel=nsrc * N), _dev(grad, "grad", numel=3 * N), int(acc),
                             _dev(ws, "ws", torch.uint8), ws.numel(), _stream(dev)))
    return grad


def kernel_density(grid, s, dens, grad, eps, zeta):
    """Kernel-density normalisation (Eqs. (18)-(19)): returns (K [3, *n], Kd [*n])
    from dens (s-gradient row of tt_kernel over the R = 1 adjoint fields) and the
    summed misfit gradients grad [3, *n]."""
    lib = _lib.load()
    N = _N(grid)
    dev = s.device
    K = torch.empty((3,) + tuple(int(v) for v in grid["n"]), dtype=_F64, device=dev)
    Kd = torch.empty(tuple(int(v) for v in grid["n"]), dtype=_F64, device=dev)
    g = _grid(grid)
    _lib.check(lib.tt_kernel_density(ctypes.byref(g), _dev(s, "s", numel=N), _dev(dens, "dens", numel=N),
                                     _dev(grad, "grad", numel=3 * N), float(eps), float(zeta), _dev(K, "K"),
                                     _dev(Kd, "Kd"), _stream(dev)))
    return K, Kd


def _mg_args(inv_grids, device):
    """(m host int32 array, coords device tensor, per-grid sizes) of inversion
    grids given as [(r, theta, phi), ...] ascending coordinate sequences."""
    sizes = [tuple(len(c) for c in axes) for axes in inv_grids]
    m = (ctypes.c_int32 * (3 * len(inv_grids)))(*[v for sz in sizes for v in sz])
    flat = [float(v) for axes in inv_grids for c in axes for v in (c.tolist() if hasattr(c, "tolist") else c)]
    coords = torch.tensor(flat, dtype=_F64, device=device)
    return m, coords, sizes


def mg_workspace_size(grid, inv_grids):
    """Bytes of workspace tt_mg_project needs for these inversion grids (0: the
    one-wave-per-node form, no workspace)."""
    lib = _lib.load()
    sizes = [tuple(len(c) for c in axes) for axes in inv_grids]
    m = (ctypes.c_int32 * (3 * len(sizes)))(*[v for sz in sizes for v in sz])
    g = _grid(grid)
    return int(lib.tt_mg_workspace_size(ctypes.byref(g), len(sizes), m))


def mg_project(grid, inv_grids, K):
    """d chi / d C (Eq. (17)) on each inversion grid: list of [3, m0, m1, m2] tensors."""
    lib = _lib.load()
    dev = K.device
    m, coords, sizes = _mg_args(inv_grids, dev)
    total = sum(3 * a * b * c for a, b, c in sizes)
    out = torch.empty(total, dtype=_F64, device=dev)
    g = _grid(grid)
    nws = int(lib.tt_mg_workspace_size(ctypes.byref(g), len(inv_grids), m))
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
    _lib.check(lib.tt_mg_project(ctypes.byref(g), len(inv_grids), m, _dev(coords, "coords"),
                                 _dev(K, "K", numel=3 * _N(grid)), _dev(out, "out"),
                                 _dev(ws, "ws", torch.uint8), ctypes.c_size_t(nws), _stream(dev)))
    res, off = [], 0
    for sz in sizes:
        n = 3 * sz[0] * sz[1] * sz[2]
        res.append(out[off:off + n].view((3,) + sz))
        off += n
    return res


def mg_expand(grid, inv_grids, C):
    """Fields [3, *n] = sum of C B over the inversion grids (Eq. (15)); C is a
    list of [3, m0, m1, m2] tensors."""
    lib = _lib.load()
    dev = C[0].device
    m, coords, sizes = _mg_args(inv_grids, dev)
    Cf = torch.cat([c.reshape(-1) for c in C]).contiguous()
    field = torch.empty((3,) + tuple(int(v) for v in grid["n"]), dtype=_F64, device=dev)
    g = _grid(grid)
    _lib.check(lib.tt_mg_expand(ctypes.byref(g), len(inv_grids), m, _dev(coords, "coords"), _dev(Cf, "C"),
                                _dev(field, "field"), _stream(dev)))
    return field
