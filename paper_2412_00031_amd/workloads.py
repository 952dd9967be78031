"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module holds no arithmetic of the method itself (no traveltimes, no
sweeps, no interpolation of the model at sources): only grids, model fields,
source/receiver positions, pair lists, residuals and observation stand-ins.
All outputs are numpy float64 (positions in axis coordinates: km for r/z/y/x,
radians for latitude/longitude).

Workloads (the paper has no public dataset for this path; these stand in for
the synthetic set-ups of its Sec. 3 and the grid sizes of its Table 1 and
Sec. 4):

* ``cartesian41``  41^3 Cartesian, h = 1 km, v = 6 + 0.02 z km/s, isotropic,
  one source uniform in [1, 39]^3 km, 20 receivers on random surface nodes,
  residuals R ~ N(0, 0.1^2) s, tol 1e-8.
* ``sph61``        61^3 spherical, depth 0-60 km, latitude/longitude in
  [-1 deg, 1 deg]; 1-D velocity 5.5 -> 7.5 km/s with depth times a +-5 %
  smooth checkerboard of 10 km cells; xi, eta = 0.03 cos/sin(2 psi) with psi
  uniform on [0, pi) per 10 km cell; 32 sources at depth U(5, 40) km in the
  central 80 % laterally; 200 receivers on distinct surface nodes.
* ``sph61_batch``  as ``sph61`` with 256 sources at depth U(1, 55) km and 2000
  distinct unordered receiver pairs.
* ``sph101``       101^3 spherical, depth 0-100 km, [-2 deg, 2 deg]^2;
  background v = 6 + 0.02 d; s = s_bg (1 + 0.1 g_s), xi = 0.04 g_xi,
  eta = 0.04 g_eta with Gaussian random fields of 10 km correlation length
  (FFT filtering, normalised to max |g| = 1); 128 sources at depth U(5, 90) km
  in the central 80 %; 500 receivers on distinct surface nodes.
"""
import math

import numpy as np

R_EARTH = 6371.0
DEG = math.pi / 180.0


def cartesian_grid(n, h):
    return dict(n=(n, n, n), coord=0, o=(0.0, 0.0, 0.0), h=(h, h, h))


def spherical_grid(n, depth_km, half_width_deg, n_lat=None, n_lon=None):
    """r ascends with the first index (surface at i = n-1); angles centred on 0."""
    n1 = n_lat or n
    n2 = n_lon or n
    hr = depth_km / (n - 1)
    ha = 2.0 * half_width_deg * DEG / (n1 - 1)
    hb = 2.0 * half_width_deg * DEG / (n2 - 1)
    return dict(n=(n, n1, n2), coord=1, o=(R_EARTH - depth_km, -half_width_deg * DEG, -half_width_deg * DEG),
                h=(hr, ha, hb))


def axes(grid):
    return [grid["o"][a] + grid["h"][a] * np.arange(grid["n"][a]) for a in range(3)]


def depth_of(grid):
    """Depth (km) of each first-axis index."""
    x0 = axes(grid)[0]
    return (R_EARTH - x0) if grid["coord"] == 1 else x0


def surface_index(grid):
    return grid["n"][0] - 1 if grid["coord"] == 1 else 0


def _arc_km(grid):
    """Surface arc lengths (km) of the two lateral axes from the domain corner."""
    ax = axes(grid)
    if grid["coord"] == 1:
        return (ax[1] - ax[1][0]) * R_EARTH, (ax[2] - ax[2][0]) * R_EARTH
    return ax[1] - ax[1][0], ax[2] - ax[2][0]


def gaussian_random_field(shape, spacing_km, corr_km, rng):
    """Zero-mean field with covariance ~ exp(-r^2 / (2 corr^2)) by FFT filtering,
    normalised to max |g| = 1."""
    white = rng.standard_normal(shape)
    ks = [np.fft.fftfreq(shape[a], d=spacing_km[a]) * 2.0 * math.pi for a in range(3)]
    K2 = ks[0][:, None, None] ** 2 + ks[1][None, :, None] ** 2 + ks[2][None, None, :] ** 2
    filt = np.exp(-0.25 * K2 * corr_km * corr_km)
    g = np.real(np.fft.ifftn(np.fft.fftn(white) * filt))
    g -= g.mean()
    return g / np.abs(g).max()


def grid_spacing_km(grid):
    if grid["coord"] == 1:
        return (grid["h"][0], grid["h"][1] * R_EARTH, grid["h"][2] * R_EARTH)
    return tuple(grid["h"])


def random_surface_nodes(grid, count, rng):
    n1, n2 = grid["n"][1], grid["n"][2]
    flat = rng.choice(n1 * n2, size=count, replace=False)
    ax = axes(grid)
    j, k = flat // n2, flat % n2
    i = surface_index(grid)
    return np.stack([np.full(count, ax[0][i]), ax[1][j], ax[2][k]], axis=1)


def random_sources(grid, count, depth_range, rng, lateral_frac=0.8):
    ax = axes(grid)
    d = rng.uniform(depth_range[0], depth_range[1], count)
    x0 = (R_EARTH - d) if grid["coord"] == 1 else d
    out = [x0]
    for a in (1, 2):
        lo, hi = ax[a][0], ax[a][-1]
        c, half = 0.5 * (lo + hi), 0.5 * (hi - lo) * lateral_frac
        out.append(rng.uniform(c - half, c + half, count))
    return np.stack(out, axis=1)


def random_pairs(nrec, count, rng):
    """Distinct unordered receiver pairs (m, i), m < i."""
    seen = set()
    out = []
    while len(out) < count:
        m, i = rng.integers(0, nrec, 2)
        if m == i:
            continue
        key = (min(m, i), max(m, i))
        if key in seen:
            continue
        seen.add(key)
        out.append(key)
    return np.asarray(out, dtype=np.int32)


def staggered_inversion_grids(grid, m, H):
    """H regular inversion grids of m = (m0, m1, m2) nodes each, spacing
    d_a = span_a / (m_a - 2), grid h shifted by h d_a / H along every axis, so
    each covers the forward grid and the H grids interleave (the
    multiple-grid parameterisation of Eqs. (11)-(17))."""
    ax = axes(grid)
    out = []
    for h in range(H):
        g = []
        for a in range(3):
            lo, hi = ax[a][0], ax[a][-1]
            d = (hi - lo) / (m[a] - 2)
            g.append(lo - d + d * h / H + d * np.arange(m[a]))
        out.append(tuple(g))
    return out


def receiver_source_pairs(nsrc, nrec, per_rec, rng):
    """Common-receiver pairs grouped by receiver: per_rec distinct unordered
    source pairs (n, j), n < j, at each receiver (fewer if nsrc is small).
    Returns (off [nrec+1], pair [off[-1], 2]) int32 and the same pairs as
    triples (n, j, m) [off[-1], 3] in the same order."""
    off = [0]
    pair = []
    for _ in range(nrec):
        cnt = min(per_rec, nsrc * (nsrc - 1) // 2)
        seen = set()
        while len(seen) < cnt:
            n, j = rng.integers(0, nsrc, 2)
            if n == j or (min(n, j), max(n, j)) in seen:
                continue
            seen.add((min(n, j), max(n, j)))
            pair.append((min(n, j), max(n, j)))
        off.append(len(pair))
    off = np.asarray(off, dtype=np.int32)
    pair = np.asarray(pair, dtype=np.int32).reshape(-1, 2)
    m = np.repeat(np.arange(nrec, dtype=np.int32), np.diff(off))
    return off, pair, np.concatenate([pair, m[:, None]], axis=1)


def straight_line_times(grid, src_pos, rec_pos, v_ref):
    """Observation stand-ins: straight-chord distance / v_ref (km/s).  A data
    generator only (no relation to the solver's discretisation)."""
    def embed(p):
        p = np.asarray(p, dtype=np.float64)
        if grid["coord"] == 0:
            return p
        r, th, ph = p[..., 0], p[..., 1], p[..., 2]
        return np.stack([r * np.cos(th) * np.cos(ph), r * np.cos(th) * np.sin(ph), r * np.sin(th)], -1)
    S = embed(src_pos)[:, None, :]
    Rr = embed(rec_pos)[None, :, :]
    return np.linalg.norm(Rr - S, axis=-1) / v_ref


def cartesian41(seed=1001, n=41, h=1.0):
    rng = np.random.default_rng(seed)
    grid = cartesian_grid(n, h)
    z = axes(grid)[0]
    v = 6.0 + 0.02 * z
    s = np.broadcast_to((1.0 / v)[:, None, None], grid["n"]).copy()
    xi = np.zeros(grid["n"])
    eta = np.zeros(grid["n"])
    L = (n - 1) * h
    src = rng.uniform(0.025 * L, 0.975 * L, (1, 3))
    rec = random_surface_nodes(grid, 20, rng)
    R = rng.normal(0.0, 0.1, (1, 20))
    return dict(name="cartesian41", grid=grid, s=s, xi=xi, eta=eta, src=src, rec=rec, R=R,
                kappa=1.0, tol=1e-8, pairs=None)


def _sph61_model(grid, rng):
    d = depth_of(grid)
    v1 = 5.5 + 2.0 * d / 60.0
    y, x = _arc_km(grid)
    cb = (np.sin(math.pi * d / 10.0)[:, None, None] * np.sin(math.pi * y / 10.0)[None, :, None]
          * np.sin(math.pi * x / 10.0)[None, None, :])
    v = v1[:, None, None] * (1.0 + 0.05 * cb)
    s = 1.0 / v
    # psi uniform on [0, pi) per 10 km cell
    ci = np.floor(d / 10.0).astype(int)
    cj = np.floor(y / 10.0).astype(int)
    ck = np.floor(x / 10.0).astype(int)
    psi_cells = rng.uniform(0.0, math.pi, (ci.max() + 1, cj.max() + 1, ck.max() + 1))
    psi = psi_cells[ci[:, None, None], cj[None, :, None], ck[None, None, :]]
    xi = 0.03 * np.cos(2.0 * psi)
    eta = 0.03 * np.sin(2.0 * psi)
    s_bg = np.broadcast_to((1.0 / v1)[:, None, None], grid["n"]).copy()
    return s, xi, eta, s_bg


def sph61(seed=2001, n=61, nsrc=32, nrec=200):
    rng = np.random.default_rng(seed)
    grid = spherical_grid(n, 60.0, 1.0)
    s, xi, eta, _ = _sph61_model(grid, rng)
    src = random_sources(grid, nsrc, (5.0, 40.0), rng)
    rec = random_surface_nodes(grid, nrec, rng)
    R = rng.normal(0.0, 0.1, (nsrc, nrec))
    return dict(name="sph61", grid=grid, s=s, xi=xi, eta=eta, src=src, rec=rec, R=R,
                kappa=1.05, tol=1e-6, pairs=None)


def sph61_batch(seed=3001, n=61, nsrc=256, nrec=200, npair=2000):
    rng = np.random.default_rng(seed)
    grid = spherical_grid(n, 60.0, 1.0)
    s, xi, eta, s_bg = _sph61_model(grid, rng)
    src = random_sources(grid, nsrc, (1.0, 55.0), rng)
    rec = random_surface_nodes(grid, nrec, rng)
    pairs = random_pairs(nrec, npair, rng)
    return dict(name="sph61_batch", grid=grid, s=s_bg, xi=np.zeros(grid["n"]), eta=np.zeros(grid["n"]),
                s_true=s, xi_true=xi, eta_true=eta, src=src, rec=rec, pairs=pairs,
                kappa=1.05, tol=1e-6)


def _grf_model(grid, rng):
    d = depth_of(grid)
    s_bg = (1.0 / (6.0 + 0.02 * d))[:, None, None]
    sp = grid_spacing_km(grid)
    gs = gaussian_random_field(grid["n"], sp, 10.0, rng)
    gx = gaussian_random_field(grid["n"], sp, 10.0, rng)
    ge = gaussian_random_field(grid["n"], sp, 10.0, rng)
    s = np.ascontiguousarray(s_bg * (1.0 + 0.1 * gs))
    return s, 0.04 * gx, 0.04 * ge


def sph101(seed=4001, n=101, nsrc=128, nrec=500, with_true=True):
    rng = np.random.default_rng(seed)
    grid = spherical_grid(n, 100.0, 2.0)
    s, xi, eta = _grf_model(grid, rng)
    src = random_sources(grid, nsrc, (5.0, 90.0), rng)
    rec = random_surface_nodes(grid, nrec, rng)
    out = dict(name="sph101", grid=grid, s=s, xi=xi, eta=eta, src=src, rec=rec,
               kappa=1.05, tol=1e-6, pairs=None)
    if with_true:
        rt = np.random.default_rng(seed + 100)
        st, xt, et = _grf_model(grid, rt)
        out.update(s_true=st, xi_true=xt, eta_true=et)
    out["R"] = np.random.default_rng(seed + 7).normal(0.0, 0.1, (nsrc, nrec))
    return out


def sph121(seed=5001, n=121, nsrc=512):
    """Evaluation workload of the learned warm start: the 0-100 km, 4 x 4 degree
    spherical box of sph101 on a finer 121^3 grid (h = 0.83 km), a GRF model of
    the same statistics (never trained on) and 512 sources at 5-90 km."""
    rng = np.random.default_rng(seed)
    grid = spherical_grid(n, 100.0, 2.0)
    s, xi, eta = _grf_model(grid, rng)
    src = random_sources(grid, nsrc, (5.0, 90.0), rng)
    return dict(name="sph121", grid=grid, s=s, xi=xi, eta=eta, src=src, kappa=1.05, tol=1e-6)


def small_spherical(n=(13, 14, 15), depth_km=12.0, half_width_deg=0.12, seed=7, aniso=0.03, nsrc=2,
                    nrec=9):
    """Tiny spherical case with a smooth anisotropic model (several tiles and
    ragged tails at small sizes)."""
    rng = np.random.default_rng(seed)
    grid = spherical_grid(n[0], depth_km, half_width_deg, n_lat=n[1], n_lon=n[2])
    d = depth_of(grid)
    y, x = _arc_km(grid)
    v = (6.0 + 0.05 * d)[:, None, None] * (1.0 + 0.04 * np.sin(0.7 * y)[None, :, None]
                                           * np.cos(0.5 * x)[None, None, :])
    s = 1.0 / v
    xi = aniso * np.cos(0.3 * d)[:, None, None] * np.cos(0.4 * y)[None, :, None] * np.ones(grid["n"])
    eta = aniso * np.sin(0.25 * x)[None, None, :] * np.ones(grid["n"])
    src = random_sources(grid, nsrc, (0.2 * depth_km, 0.8 * depth_km), rng)
    rec = random_surface_nodes(grid, nrec, rng)
    R = rng.normal(0.0, 0.1, (nsrc, nrec))
    return dict(name="small_spherical", grid=grid, s=np.ascontiguousarray(s), xi=np.ascontiguousarray(xi),
                eta=np.ascontiguousarray(eta), src=src, rec=rec, R=R, kappa=1.05, tol=1e-10, pairs=None)
