"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``oracle.c`` (see its header for the
equations and readings it follows) with ctypes over numpy arrays, and adds the
tiny-grid numpy tools in :mod:`oracle.tiny`.

Grid description used throughout: a mapping with keys ``n`` (3 ints),
``coord`` (0 Cartesian z/y/x in km, 1 spherical r km / latitude rad /
longitude rad), ``o`` and ``h`` (3 floats each).  Fields are numpy float64
arrays of shape ``n`` (axis 2 fastest).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = ctypes.CDLL(path)
        _lib.tto_misfit.restype = ctypes.c_double
        _lib.tto_misfit_cr.restype = ctypes.c_double
        _lib.tto_lf_update.restype = ctypes.c_double
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle needs contiguous float64"
    return a.ctypes.data_as(_D)


def _i(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_I)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid_args(grid):
    n = np.asarray(grid["n"], dtype=np.int32)
    o = np.asarray(grid["o"], dtype=np.float64)
    h = np.asarray(grid["h"], dtype=np.float64)
    return n, int(grid["coord"]), o, h


def _shape(grid):
    return tuple(int(v) for v in grid["n"])


def source_params(grid, s, xi, eta, src_pos):
    """s0, xi0, eta0 at each source: trilinear interpolation of the model."""
    n, coord, o, h = _grid_args(grid)
    src_pos = _f64(src_pos).reshape(-1, 3)
    out = np.zeros_like(src_pos)
    rc = lib().tto_source_params(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(xi)), _d(_f64(eta)),
                                 len(src_pos), _d(src_pos), _d(out))
    if rc:
        raise ValueError("source outside the grid")
    return out


def forward(grid, s, xi, eta, src_pos, src_par, kappa, tol, max_iter, order=0, tau_init=None):
    """One-source forward solve.  Returns (tau, iters, converged, eps_history)."""
    n, coord, o, h = _grid_args(grid)
    tau = np.empty(_shape(grid), dtype=np.float64)
    iters, conv = ctypes.c_int(0), ctypes.c_int(0)
    hist = np.zeros(max_iter, dtype=np.float64)
    rc = lib().tto_forward(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(xi)), _d(_f64(eta)),
                           _d(_f64(src_pos)), _d(_f64(src_par)), ctypes.c_double(kappa),
                           ctypes.c_double(tol), int(max_iter), int(order),
                           _d(_f64(tau_init)) if tau_init is not None else None, _d(tau),
                           ctypes.byref(iters), ctypes.byref(conv), _d(hist))
    if rc:
        raise ValueError("invalid arguments")
    return tau, iters.value, bool(conv.value), hist[: iters.value].copy()


def lf_update(grid, s, xi, eta, src_pos, src_par, kappa, tau, i, j, k):
    n, coord, o, h = _grid_args(grid)
    return lib().tto_lf_update(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(xi)), _d(_f64(eta)),
                               _d(_f64(src_pos)), _d(_f64(src_par)), ctypes.c_double(kappa),
                               _d(_f64(tau)), int(i), int(j), int(k))


def factor_field(grid, src_pos, src_par):
    """T0 [n] and its scaled gradient t [3, n]."""
    n, coord, o, h = _grid_args(grid)
    T0 = np.empty(_shape(grid))
    t = np.empty((3,) + _shape(grid))
    lib().tto_factor_field(_i(n), coord, _d(o), _d(h), _d(_f64(src_pos)), _d(_f64(src_par)), _d(T0), _d(t))
    return T0, t


def fixed_base(grid, src_pos):
    n, coord, o, h = _grid_args(grid)
    fb = np.zeros(3, dtype=np.int32)
    lib().tto_fixed_base(_i(n), coord, _d(o), _d(h), _d(_f64(src_pos)), _i(fb))
    return tuple(int(v) for v in fb)


def sample(grid, src_pos, src_par, tau, rec_pos):
    """T at receivers for one source."""
    n, coord, o, h = _grid_args(grid)
    rec_pos = _f64(rec_pos).reshape(-1, 3)
    out = np.zeros(len(rec_pos))
    rc = lib().tto_sample(_i(n), coord, _d(o), _d(h), _d(_f64(src_pos)), _d(_f64(src_par)), _d(_f64(tau)),
                          len(rec_pos), _d(rec_pos), _d(out))
    if rc:
        raise ValueError("receiver outside the grid")
    return out


def misfit(T, T_obs, w=None, pairs=None, wpair=None, alpha=1.0, beta=1.0):
    """chi and R = d chi / d T for [nsrc, nrec] traveltimes."""
    T = _f64(T)
    nsrc, nrec = T.shape
    R = np.zeros_like(T)
    if pairs is None:
        pairs_a = np.zeros((0, 2), dtype=np.int32)
    else:
        pairs_a = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    chi = lib().tto_misfit(nsrc, nrec, _d(T), _d(_f64(T_obs)), _d(_f64(w)) if w is not None else None,
                           len(pairs_a), _i(pairs_a), _d(_f64(wpair)) if wpair is not None else None,
                           ctypes.c_double(alpha), ctypes.c_double(beta), _d(R))
    return chi, R


def misfit_cr(T, T_obs, tri, wtri=None, gamma=1.0, R=None):
    """gamma * chi_cr (Eq. (4)) for source-pair triples tri [ntri, 3] = (n, j, m),
    each unordered pair at a receiver listed once; adds d chi_cr / d T (Eq. (A4))
    to R (zeros if None).  Returns (chi_cr, R)."""
    T = _f64(T)
    nsrc, nrec = T.shape
    R = np.zeros_like(T) if R is None else np.ascontiguousarray(R, dtype=np.float64)
    tri_a = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    chi = lib().tto_misfit_cr(nsrc, nrec, _d(T), _d(_f64(T_obs)), len(tri_a), _i(tri_a),
                              _d(_f64(wtri)) if wtri is not None else None, ctypes.c_double(gamma), _d(R))
    if np.isnan(chi):
        raise ValueError("common-receiver triple index out of range")
    return chi, R


def adjoint_rhs(grid, src_pos, src_par, rec_pos, R):
    n, coord, o, h = _grid_args(grid)
    rec_pos = _f64(rec_pos).reshape(-1, 3)
    g = np.zeros(_shape(grid))
    rc = lib().tto_adjoint_rhs(_i(n), coord, _d(o), _d(h), _d(_f64(src_pos)), _d(_f64(src_par)),
                               len(rec_pos), _d(rec_pos), _d(_f64(R)), _d(g))
    if rc:
        raise ValueError("receiver outside the grid")
    return g


def adjoint_coeffs(grid, s, xi, eta, src_pos, src_par, kappa, tau):
    """[7, n]: alpha_0..2, beta_0..2, J_xx at interior non-fixed nodes."""
    n, coord, o, h = _grid_args(grid)
    out = np.zeros((7,) + _shape(grid))
    lib().tto_adjoint_coeffs(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(xi)), _d(_f64(eta)),
                             _d(_f64(src_pos)), _d(_f64(src_par)), ctypes.c_double(kappa), _d(_f64(tau)), _d(out))
    return out


def adjoint(grid, s, xi, eta, src_pos, src_par, kappa, tau, rhs, tol, max_iter, order=0):
    """Solve J^T lambda = rhs by transposed Gauss-Seidel sweeps.
    Returns (lambda, iters, converged, eps_history)."""
    n, coord, o, h = _grid_args(grid)
    lam = np.zeros(_shape(grid))
    iters, conv = ctypes.c_int(0), ctypes.c_int(0)
    hist = np.zeros(max_iter)
    rc = lib().tto_adjoint(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(xi)), _d(_f64(eta)),
                           _d(_f64(src_pos)), _d(_f64(src_par)), ctypes.c_double(kappa), _d(_f64(tau)),
                           _d(_f64(rhs)), ctypes.c_double(tol), int(max_iter), int(order), _d(lam),
                           ctypes.byref(iters), ctypes.byref(conv), _d(hist))
    if rc:
        raise ValueError("invalid arguments")
    return lam, iters.value, bool(conv.value), hist[: iters.value].copy()


def reloc_times(grid, field_pos, field_par, tau, ev_pos, ev_t0=None):
    """T [nev, nfield] = Gamma_m(x_n) + t_n (App. B): field m is the forward
    solution with receiver m as the source."""
    n, coord, o, h = _grid_args(grid)
    field_pos = _f64(field_pos).reshape(-1, 3)
    ev_pos = _f64(ev_pos).reshape(-1, 3)
    T = np.zeros((len(ev_pos), len(field_pos)))
    rc = lib().tto_reloc_times(_i(n), coord, _d(o), _d(h), len(field_pos), _d(field_pos),
                               _d(_f64(field_par).reshape(-1, 3)), _d(_f64(tau)), len(ev_pos), _d(ev_pos),
                               _d(_f64(ev_t0)) if ev_t0 is not None else None, _d(T))
    if rc:
        raise ValueError("earthquake outside the grid")
    return T


def reloc_kernel(grid, field_pos, field_par, tau, ev_pos, R):
    """Eq. (10): K [nev, 4] = (d chi/d x_0, d chi/d x_1, d chi/d x_2 of each
    earthquake in grid coordinates, d chi / d t_n) from R = d chi / d T [nev, nfield]."""
    n, coord, o, h = _grid_args(grid)
    field_pos = _f64(field_pos).reshape(-1, 3)
    ev_pos = _f64(ev_pos).reshape(-1, 3)
    K = np.zeros((len(ev_pos), 4))
    rc = lib().tto_reloc_kernel(_i(n), coord, _d(o), _d(h), len(field_pos), _d(field_pos),
                                _d(_f64(field_par).reshape(-1, 3)), _d(_f64(tau)), len(ev_pos), _d(ev_pos),
                                _d(_f64(R)), _d(K))
    if rc:
        raise ValueError("earthquake outside the grid")
    return K


def adjoint_cont(grid, s, xi, eta, src_pos, src_par, tau, rec_pos, R, tol, max_iter):
    """P of Eq. (5) by the upwind finite-volume discretisation (reading R14):
    point sources R_m at rec_pos through trilinear weights.  Returns
    (P, iters, converged, eps_history)."""
    n, coord, o, h = _grid_args(grid)
    P = np.zeros(_shape(grid))
    rec_pos = _f64(rec_pos).reshape(-1, 3)
    iters, conv = ctypes.c_int(0), ctypes.c_int(0)
    hist = np.zeros(max_iter)
    rc = lib().tto_adjoint_cont(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(xi)), _d(_f64(eta)),
                                _d(_f64(src_pos)), _d(_f64(src_par)), _d(_f64(tau)), len(rec_pos), _d(rec_pos),
                                _d(_f64(R)), ctypes.c_double(tol), int(max_iter), _d(P), ctypes.byref(iters),
                                ctypes.byref(conv), _d(hist))
    if rc:
        raise ValueError("invalid arguments or receiver outside the grid")
    return P, iters.value, bool(conv.value), hist[: iters.value].copy()


def cont_velocity(grid, xi, eta, src_pos, src_par, tau):
    """The transport velocity w = -M grad T [3, n] of the continuous adjoint
    (reading R14) for a given tau: central differences of tau on interior
    axes, one-sided on boundary axes."""
    n, coord, o, h = _grid_args(grid)
    w = np.empty((3,) + _shape(grid))
    rc = lib().tto_cont_velocity(_i(n), coord, _d(o), _d(h), _d(_f64(xi)), _d(_f64(eta)), _d(_f64(src_pos)),
                                 _d(_f64(src_par)), _d(_f64(tau)), _d(w))
    if rc:
        raise ValueError("invalid grid")
    return w


def kernel(grid, s, xi, eta, src_pos, src_par, kappa, tau, lam, grad=None):
    """Discrete gradients [3, n] (d chi/d s, d chi/d xi, d chi/d eta); adds to grad if given."""
    n, coord, o, h = _grid_args(grid)
    acc = grad is not None
    if grad is None:
        grad = np.zeros((3,) + _shape(grid))
    lib().tto_kernel(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(xi)), _d(_f64(eta)),
                     _d(_f64(src_pos)), _d(_f64(src_par)), ctypes.c_double(kappa), _d(_f64(tau)),
                     _d(_f64(lam)), _d(grad), int(acc))
    return grad


def node_volume(grid):
    n, coord, o, h = _grid_args(grid)
    V = np.zeros(_shape(grid))
    lib().tto_node_volume(_i(n), coord, _d(o), _d(h), _d(V))
    return V


def kernel_density(grid, s, dens, grad, eps, zeta):
    """(K [3, n], Kd [n]): paper kernels K_s, K_xi, K_eta of the summed discrete
    gradients grad [3, n], normalised by the kernel density Kd made from dens,
    the summed s-gradient of the R = 1 adjoint fields (Eqs. (18)-(19)); see
    oracle.c."""
    n, coord, o, h = _grid_args(grid)
    K = np.zeros((3,) + _shape(grid))
    Kd = np.zeros(_shape(grid))
    lib().tto_kernel_density(_i(n), coord, _d(o), _d(h), _d(_f64(s)), _d(_f64(dens)), _d(_f64(grad)),
                             ctypes.c_double(eps), ctypes.c_double(zeta), _d(K), _d(Kd))
    return K, Kd


def _mg_args(inv_grids):
    m = np.array([[len(c) for c in axes] for axes in inv_grids], dtype=np.int32).reshape(-1)
    coords = np.concatenate([np.asarray(c, dtype=np.float64) for axes in inv_grids for c in axes])
    sizes = [int(np.prod([len(c) for c in axes])) for axes in inv_grids]
    return m, coords, sizes


def mg_project(grid, inv_grids, K):
    """d chi / d C (Eq. (17)) for inversion grids inv_grids = [(r, th, ph), ...]
    (ascending coordinate arrays): list of [3, m0, m1, m2] arrays, one per grid."""
    n, coord, o, h = _grid_args(grid)
    m, coords, sizes = _mg_args(inv_grids)
    out = np.zeros(3 * sum(sizes))
    lib().tto_mg_project(_i(n), coord, _d(o), _d(h), len(inv_grids), m.ctypes.data_as(_I), _d(coords),
                         _d(_f64(K)), _d(out))
    res, off = [], 0
    for axes, sz in zip(inv_grids, sizes):
        res.append(out[off:off + 3 * sz].reshape((3,) + tuple(len(c) for c in axes)))
        off += 3 * sz
    return res


def mg_expand(grid, inv_grids, C):
    """Fields [3, n] = sum over grids and basis functions of C B (Eq. (15));
    C: list of [3, m0, m1, m2] arrays, one per grid."""
    n, coord, o, h = _grid_args(grid)
    m, coords, sizes = _mg_args(inv_grids)
    Cf = np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for c in C])
    field = np.zeros((3,) + _shape(grid))
    lib().tto_mg_expand(_i(n), coord, _d(o), _d(h), len(inv_grids), m.ctypes.data_as(_I), _d(coords), _d(Cf),
                        _d(field))
    return field


def solve_source(grid, s, xi, eta, src_pos, src_par, kappa, rec_pos, T_obs=None, R=None,
                 tol=1e-6, adj_tol=None, max_iter=2000, w=None):
    """Forward + sample + (misfit) + adjoint + kernel for one source (chi_t only).
    Returns a dict with tau, T_rec, R, lam, grad and iteration counts."""
    tau, it_f, cf, _ = forward(grid, s, xi, eta, src_pos, src_par, kappa, tol, max_iter)
    T_rec = sample(grid, src_pos, src_par, tau, rec_pos)
    chi = None
    if R is None:
        chi, Rm = misfit(T_rec[None, :], np.asarray(T_obs)[None, :], None if w is None else np.asarray(w)[None, :])
        R = Rm[0]
    g = adjoint_rhs(grid, src_pos, src_par, rec_pos, R)
    lam, it_a, ca, _ = adjoint(grid, s, xi, eta, src_pos, src_par, kappa, tau, g,
                               adj_tol if adj_tol is not None else tol, max_iter)
    grad = kernel(grid, s, xi, eta, src_pos, src_par, kappa, tau, lam)
    return dict(tau=tau, T_rec=T_rec, chi=chi, R=R, lam=lam, grad=grad, it_f=it_f, it_a=it_a,
                conv_f=cf, conv_a=ca)
