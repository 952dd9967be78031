"""Tiny-grid numpy tools for pinning the oracle (test infrastructure only).

``residual`` writes out the discrete forward system that the sweeps solve
(interior Lax-Friedrichs equations, boundary copy rows, fixed rows),
vectorised in numpy; ``jacobian_fd`` differentiates it numerically.  They let
the tests check the Gauss-Seidel solvers against dense direct solves (Newton
for the forward fixed point, J^T lambda = g for the adjoint).
"""
import numpy as np

from . import factor_field, fixed_base


def _metric(grid):
    n = tuple(grid["n"])
    if grid["coord"] == 0:
        return [np.ones(n), np.ones(n), np.ones(n)]
    r = grid["o"][0] + grid["h"][0] * np.arange(n[0])
    th = grid["o"][1] + grid["h"][1] * np.arange(n[1])
    g1 = np.broadcast_to((1.0 / r)[:, None, None], n)
    g2 = np.broadcast_to((1.0 / (r[:, None] * np.cos(th)[None, :]))[:, :, None], n)
    return [np.ones(n), g1, g2]


def node_classes(grid, src_pos):
    """Boolean masks (fixed, boundary-not-fixed, interior-not-fixed)."""
    n = tuple(grid["n"])
    fb = fixed_base(grid, src_pos)
    F = np.zeros(n, dtype=bool)
    F[fb[0]:fb[0] + 2, fb[1]:fb[1] + 2, fb[2]:fb[2] + 2] = True
    B = np.zeros(n, dtype=bool)
    B[0, :, :] = B[-1, :, :] = True
    B[:, 0, :] = B[:, -1, :] = True
    B[:, :, 0] = B[:, :, -1] = True
    return F, B & ~F, ~B & ~F


def residual(grid, s, xi, eta, src_pos, src_par, kappa, tau):
    """Residual of every row of the discrete forward system (shape n)."""
    n = tuple(grid["n"])
    T0, t = factor_field(grid, src_pos, src_par)
    gm = _metric(grid)
    h = grid["h"]
    F, Bn, In = node_classes(grid, src_pos)
    res = np.zeros(n)
    # interior rows
    sl = (slice(1, -1),) * 3
    def sh(a, off):
        idx = [slice(1, -1)] * 3
        idx[a] = slice(1 + off, n[a] - 1 + off)
        return tau[tuple(idx)]
    P = []
    visc = 0.0
    for a in range(3):
        q = gm[a][sl] * (sh(a, 1) - sh(a, -1)) / (2.0 * h[a])
        P.append(T0[sl] * q + tau[sl] * t[a][sl])
        visc = visc + kappa * T0[sl] * gm[a][sl] * (sh(a, 1) - 2.0 * tau[sl] + sh(a, -1)) / (2.0 * h[a])
    x, e = xi[sl], eta[sl]
    H = np.sqrt(P[0] ** 2 + (1 - 2 * x) * P[1] ** 2 + 4 * e * P[1] * P[2] + (1 + 2 * x) * P[2] ** 2)
    Gint = H - visc - s[sl]
    res[sl] = Gint
    # boundary rows: copy of the inward neighbour along the largest boundary axis
    for idx in zip(*np.nonzero(Bn)):
        p = list(idx)
        as_ = max(a for a in range(3) if p[a] in (0, n[a] - 1))
        nu = 1 if p[as_] == 0 else -1
        p1 = list(p); p1[as_] += nu
        res[idx] = tau[idx] - tau[tuple(p1)]
    res[F] = tau[F] - 1.0
    return res


def jacobian_fd(grid, s, xi, eta, src_pos, src_par, kappa, tau, step=1e-7):
    """Dense Jacobian of ``residual`` by central differences, [N, N] (row = equation)."""
    N = tau.size
    J = np.zeros((N, N))
    flat = tau.reshape(-1).copy()
    for c in range(N):
        tp = flat.copy(); tp[c] += step
        tm = flat.copy(); tm[c] -= step
        rp = residual(grid, s, xi, eta, src_pos, src_par, kappa, tp.reshape(tau.shape))
        rm = residual(grid, s, xi, eta, src_pos, src_par, kappa, tm.reshape(tau.shape))
        J[:, c] = (rp - rm).reshape(-1) / (2.0 * step)
    return J


def assemble_jacobian(grid, coeffs, src_pos):
    """Dense Jacobian from the oracle's adjoint coefficients [7, n]."""
    n = tuple(grid["n"])
    N = int(np.prod(n))
    F, Bn, In = node_classes(grid, src_pos)
    J = np.zeros((N, N))
    st = (n[1] * n[2], n[2], 1)
    lin = lambda p: (p[0] * n[1] + p[1]) * n[2] + p[2]
    for idx in np.ndindex(*n):
        r = lin(idx)
        if F[idx]:
            J[r, r] = 1.0
        elif Bn[idx]:
            p = list(idx)
            as_ = max(a for a in range(3) if p[a] in (0, n[a] - 1))
            nu = 1 if p[as_] == 0 else -1
            J[r, r] = 1.0
            J[r, r + nu * st[as_]] += -1.0
        else:
            J[r, r] = coeffs[6][idx]
            for a in range(3):
                J[r, r + st[a]] += coeffs[a][idx] - coeffs[3 + a][idx]
                J[r, r - st[a]] += -coeffs[a][idx] - coeffs[3 + a][idx]
    return J


def newton(grid, s, xi, eta, src_pos, src_par, kappa, tau0, iters=30, tol=1e-14):
    """Newton's method on residual = 0 with the FD Jacobian (dense; tiny grids)."""
    tau = tau0.copy()
    for _ in range(iters):
        r = residual(grid, s, xi, eta, src_pos, src_par, kappa, tau).reshape(-1)
        if np.abs(r).max() < tol:
            break
        J = jacobian_fd(grid, s, xi, eta, src_pos, src_par, kappa, tau)
        tau = tau - np.linalg.solve(J, r).reshape(tau.shape)
    return tau
