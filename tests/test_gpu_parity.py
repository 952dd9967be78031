"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Both sides start from the same seeded inputs (paper_2412_00031_amd.workloads)
and run their own pipeline: source constants, forward solve, receiver
sampling, misfit/adjoint sources, adjoint solve, kernels.  Tolerances: tau and
T at receivers 1e-12 (normwise relative), adjoint fields and kernels 1e-10,
and identical iteration counts (the GPU visits the same Gauss-Seidel
dependencies as the lexicographic oracle, so only rounding differs).
"""
import numpy as np
import pytest

import oracle as O
from conftest import rel_inf
from paper_2412_00031_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_TAU = 1e-12
TOL_ADJ = 1e-10


def _dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def oracle_path(wl, tol, max_iter, R=None, T_obs=None, adj_tol=None, max_iter_adj=None, tau_init=None,
                nsrc=None):
    g, s, xi, eta = wl["grid"], wl["s"], wl["xi"], wl["eta"]
    src = wl["src"][:nsrc] if nsrc else wl["src"]
    rec = wl["rec"]
    par = O.source_params(g, s, xi, eta, src)
    taus, its, Ts = [], [], []
    for q in range(len(src)):
        ti = None if tau_init is None else tau_init[q]
        tau, it, conv, _ = O.forward(g, s, xi, eta, src[q], par[q], wl["kappa"], tol, max_iter, tau_init=ti)
        taus.append(tau)
        its.append(it if conv else -it)
        Ts.append(O.sample(g, src[q], par[q], tau, rec))
    T = np.stack(Ts)
    chi = None
    if R is None:
        chi, R = O.misfit(T, T_obs, pairs=wl.get("pairs"))
        cr = wl.get("cr")
        if cr is not None:
            chi_cr, R = O.misfit_cr(T, T_obs, cr["tri"], cr.get("w"), cr["gamma"], R)
            chi += chi_cr
    lams, ita = [], []
    grad = np.zeros((3,) + tuple(g["n"]))
    for q in range(len(src)):
        rhs = O.adjoint_rhs(g, src[q], par[q], rec, R[q])
        lam, it, conv, _ = O.adjoint(g, s, xi, eta, src[q], par[q], wl["kappa"], taus[q], rhs,
                                     adj_tol or tol, max_iter_adj or max_iter)
        lams.append(lam)
        ita.append(it if conv else -it)
        O.kernel(g, s, xi, eta, src[q], par[q], wl["kappa"], taus[q], lam, grad)
    return dict(par=par, tau=np.stack(taus), it_f=np.array(its), T=T, chi=chi, R=R, lam=np.stack(lams),
                it_a=np.array(ita), grad=grad)


def gpu_path(torch, wl, tol, max_iter, R=None, T_obs=None, adj_tol=None, max_iter_adj=None, tile_k=0,
             tau_init=None, nsrc=None, tile_k_adj=None):
    from paper_2412_00031_amd import api
    g = wl["grid"]
    s, xi, eta = (_dev(torch, wl[k]) for k in ("s", "xi", "eta"))
    src = _dev(torch, wl["src"][:nsrc] if nsrc else wl["src"])
    rec = _dev(torch, wl["rec"])
    par = api.source_params(g, s, xi, eta, src)
    ti = None if tau_init is None else _dev(torch, tau_init)
    tau, st_f = api.forward(g, s, xi, eta, src, par, tol, max_iter, wl["kappa"], tau_init=ti, tile_k=tile_k)
    T = api.sample(g, src, par, tau, rec)
    chi = None
    if R is None:
        pairs = None if wl.get("pairs") is None else _dev(torch, wl["pairs"], torch.int32)
        cr = wl.get("cr")
        kw = {}
        if cr is not None:
            kw = dict(cr=(_dev(torch, cr["off"], torch.int32), _dev(torch, cr["pair"], torch.int32)),
                      wcr=None if cr.get("w") is None else _dev(torch, cr["w"]), gamma=cr["gamma"])
        chi, Rd = api.misfit(T, _dev(torch, T_obs), pairs=pairs, **kw)
        chi = float(chi.item())
    else:
        Rd = _dev(torch, R)
    lam, st_a = api.adjoint(g, s, xi, eta, src, par, tau, rec, Rd, adj_tol or tol, max_iter_adj or max_iter,
                            wl["kappa"], tile_k=tile_k if tile_k_adj is None else tile_k_adj)
    grad = api.kernel(g, s, xi, eta, src, par, tau, lam)
    torch.cuda.synchronize()
    c = lambda t: t.cpu().numpy()
    return dict(par=c(par), tau=c(tau), it_f=c(st_f), T=c(T), chi=chi, R=c(Rd), lam=c(lam), it_a=c(st_a),
                grad=c(grad))


def assert_parity(gp, op, check_grad=True):
    assert np.array_equal(gp["it_f"], op["it_f"]), (gp["it_f"], op["it_f"])
    assert rel_inf(gp["par"], op["par"]) <= 1e-15
    assert rel_inf(gp["tau"], op["tau"]) <= TOL_TAU, rel_inf(gp["tau"], op["tau"])
    assert rel_inf(gp["T"], op["T"]) <= TOL_TAU, rel_inf(gp["T"], op["T"])
    assert np.array_equal(gp["it_a"], op["it_a"]), (gp["it_a"], op["it_a"])
    for q in range(len(op["lam"])):
        assert rel_inf(gp["lam"][q], op["lam"][q]) <= TOL_ADJ, (q, rel_inf(gp["lam"][q], op["lam"][q]))
    if check_grad:
        for c in range(3):
            if np.abs(op["grad"][c]).max() > 0:
                assert rel_inf(gp["grad"][c], op["grad"][c]) <= TOL_ADJ, (c, rel_inf(gp["grad"][c], op["grad"][c]))


def test_cartesian41_full_path(torch_cuda):
    wl = W.cartesian41()
    op = oracle_path(wl, wl["tol"], 400, R=wl["R"])
    gp = gpu_path(torch_cuda, wl, wl["tol"], 400, R=wl["R"])
    assert op["it_f"][0] > 1 and op["it_a"][0] > 1
    assert_parity(gp, op)


def test_small_spherical_several_tiles(torch_cuda):
    wl = W.small_spherical(n=(13, 14, 15), nsrc=3)
    op = oracle_path(wl, 1e-11, 400, R=wl["R"])
    for tk in (0, 4):
        gp = gpu_path(torch_cuda, wl, 1e-11, 400, R=wl["R"], tile_k=tk)
        assert_parity(gp, op)


def test_tile_shapes_bitwise(torch_cuda):
    """Any tile depth visits the same dependencies: results are bit-identical.
    The grids have ragged 8 x 8 tile columns (interior 19, 17, 21 and 27, 3, 2)
    and slab depths below, near and above the hyperplane extent of a column
    (depths up to 62 in both solves, among them every depth with a compiled
    instance)."""
    for n, seed in (((21, 19, 23), 11), ((29, 5, 4), 12)):
        wl = W.small_spherical(n=n, nsrc=2, seed=seed)
        ref = gpu_path(torch_cuda, wl, 1e-9, 200, R=wl["R"], tile_k=62, tile_k_adj=16)
        for tk, tka in ((1, 1), (2, 2), (3, 3), (5, 5), (7, 7), (8, 8), (13, 13), (21, 4), (32, 11), (48, 6),
                        (62, 9), (16, 12), (10, 14), (12, 15), (20, 28), (24, 32), (28, 40), (22, 48)):
            gp = gpu_path(torch_cuda, wl, 1e-9, 200, R=wl["R"], tile_k=tk, tile_k_adj=tka)
            for key in ("tau", "lam", "grad", "it_f", "it_a", "T"):
                assert np.array_equal(gp[key], ref[key]), (n, tk, tka, key)


def test_compiled_tile_depths_bitwise_cartesian(torch_cuda):
    """The sweeps have instances compiled for some tile depths (forward 16, 20,
    24, 28; adjoint 28, 32, 40, 48) besides the generic one: on a Cartesian grid
    (the spherical instances are covered above) each gives the generic
    instance's results bit for bit."""
    wl = W.cartesian41()
    ref = gpu_path(torch_cuda, wl, 1e-9, 200, R=wl["R"], tile_k=30, tile_k_adj=30)
    for tk, tka in ((16, 28), (20, 32), (24, 40), (28, 48)):
        gp = gpu_path(torch_cuda, wl, 1e-9, 200, R=wl["R"], tile_k=tk, tile_k_adj=tka)
        for key in ("tau", "lam", "grad", "it_f", "it_a", "T"):
            assert np.array_equal(gp[key], ref[key]), (tk, tka, key)


def test_graph_replay_matches_eager(torch_cuda):
    """Iterations replayed from a captured hipGraph give the eager results bit
    for bit; several solves in a row (each capturing and replaying its own
    graph, with eager work and synchronisations in between) all agree."""
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(15, 13, 17), nsrc=3, seed=19)
    g, kap = wl["grid"], wl["kappa"]
    s, xi, eta, src, rec, R = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "src", "rec", "R"))
    par = api.source_params(g, s, xi, eta, src)
    ref_tau, ref_st = api.forward(g, s, xi, eta, src, par, 1e-10, 200, kap, poll=True)
    ref_lam, ref_sa = api.adjoint(g, s, xi, eta, src, par, ref_tau, rec, R, 1e-10, 200, kap, poll=True)
    for rep in range(3):
        for poll in (True, False):
            tau, st = api.forward(g, s, xi, eta, src, par, 1e-10, 200, kap, graph=True, poll=poll)
            torch_cuda.cuda.synchronize()
            assert torch_cuda.equal(st, ref_st) and torch_cuda.equal(tau, ref_tau), (rep, poll)
            lam, sa = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, 1e-10, 200, kap, graph=True, poll=poll)
            torch_cuda.cuda.synchronize()
            assert torch_cuda.equal(sa, ref_sa) and torch_cuda.equal(lam, ref_lam), (rep, poll)
            _ = (tau * 2.0).sum().item()  # eager work between replays


def test_source_groups_bitwise(torch_cuda):
    """Splitting the batch into concurrently iterated source groups (uneven
    group sizes included, graph replay included) changes nothing: fields,
    statuses and convergence histories are bit-identical to one group, and the
    oracle agrees as for the unsplit batch."""
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(14, 15, 16), nsrc=7, nrec=10, seed=23)
    g, kap = wl["grid"], wl["kappa"]
    s, xi, eta, src, rec, R = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "src", "rec", "R"))
    par = api.source_params(g, s, xi, eta, src)

    def run(groups, graph=False, poll=False):
        hf = torch_cuda.zeros((7, 300), dtype=torch_cuda.float64, device="cuda")
        ha = torch_cuda.zeros((7, 300), dtype=torch_cuda.float64, device="cuda")
        tau, st = api.forward(g, s, xi, eta, src, par, 1e-10, 300, kap, groups=groups, eps_hist=hf, graph=graph,
                              poll=poll)
        lam, sa = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, 1e-10, 300, kap, groups=groups, eps_hist=ha,
                              graph=graph, poll=poll)
        torch_cuda.cuda.synchronize()
        return [x.cpu().numpy() for x in (tau, st, hf, lam, sa, ha)]

    ref = run(1)
    for groups, graph, poll in ((2, False, False), (3, False, True), (7, False, False), (3, True, False),
                                (3, True, True), (0, False, True), (1, False, True)):
        got = run(groups, graph, poll)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (groups, graph, poll)
    o = oracle_path(wl, 1e-10, 300, R=wl["R"])
    assert np.array_equal(ref[1], o["it_f"]) and np.array_equal(ref[4], o["it_a"])
    assert rel_inf(ref[0], o["tau"]) <= TOL_TAU and rel_inf(ref[3], o["lam"]) <= TOL_ADJ


def test_per_source_budgets(torch_cuda):
    """Per-source iteration budgets: each source group iterates the largest
    budget of its sources.  Budgets at or above every source's own count
    change nothing (fields, statuses and convergence histories bit-identical
    to a uniform budget, asynchronous and polled, several groupings); a group
    whose budgets all fall short reports -budget for its sources while the
    other group converges as before; out-of-range budgets are refused."""
    from paper_2412_00031_amd import _lib, api
    wl = W.small_spherical(n=(14, 15, 16), nsrc=6, nrec=10, seed=29)
    g, kap = wl["grid"], wl["kappa"]
    s, xi, eta, src, rec, R = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "src", "rec", "R"))
    par = api.source_params(g, s, xi, eta, src)

    def run(bf, ba, groups, poll):
        hf = torch_cuda.zeros((6, 300), dtype=torch_cuda.float64, device="cuda")
        ha = torch_cuda.zeros((6, 300), dtype=torch_cuda.float64, device="cuda")
        tau, st = api.forward(g, s, xi, eta, src, par, 1e-10, 300, kap, groups=groups, eps_hist=hf, poll=poll,
                              budgets=bf)
        lam, sa = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, 1e-10, 300, kap, groups=groups, eps_hist=ha,
                              poll=poll, budgets=ba)
        torch_cuda.cuda.synchronize()
        return [x.cpu().numpy() for x in (tau, st, hf, lam, sa, ha)]

    ref = run(None, None, 1, False)
    cf, ca = ref[1], ref[4]
    assert (cf > 0).all() and (ca > 0).all()
    for groups, poll, extra in ((2, False, 0), (3, True, 0), (1, False, 0), (6, False, 2), (2, True, 5)):
        got = run(cf + extra, ca + extra, groups, poll)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (groups, poll, extra)
    # two groups of three: the second group's budgets are all 1
    short = cf.copy()
    short[3:] = 1
    tau2, st2 = api.forward(g, s, xi, eta, src, par, 1e-10, 300, kap, groups=2, budgets=short)
    torch_cuda.cuda.synchronize()
    st2 = st2.cpu().numpy()
    assert np.array_equal(st2[:3], cf[:3]) and (st2[3:] == -1).all(), st2
    assert np.array_equal(tau2.cpu().numpy()[:3], ref[0][:3])
    for bad in ([0] + [5] * 5, [301] + [5] * 5):
        with pytest.raises(_lib.TTError):
            api.forward(g, s, xi, eta, src, par, 1e-10, 300, kap, budgets=bad)
    with pytest.raises(ValueError):
        api.forward(g, s, xi, eta, src, par, 1e-10, 300, kap, budgets=[5] * 5)


def test_compact_adjoint_records_bitwise(torch_cuda):
    """The compact record layout (one node-order copy of the adjoint's
    coefficient records, TT_FLAG_COMPACT_ADJOINT) reads the same couplings in
    the same order: discrete and continuous adjoint fields and statuses equal
    the row-layout run bit for bit at several tile depths and groupings (the
    convergence histories too at the same tile depth; other depths sum the
    per-tile partial sums in another grouping), and the oracle agrees."""
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(21, 19, 23), nsrc=5, nrec=10, seed=27)
    g, kap = wl["grid"], wl["kappa"]
    s, xi, eta, src, rec, R = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "src", "rec", "R"))
    par = api.source_params(g, s, xi, eta, src)
    tau, st = api.forward(g, s, xi, eta, src, par, 1e-11, 300, kap)
    for continuous in (False, True):
        Rc = R.abs() + 0.05 if continuous else R
        ref = None
        for compact, tk, groups in ((False, 0, 0), (True, 0, 0), (True, 5, 2), (True, 24, 1), (True, 62, 3)):
            h = torch_cuda.zeros((5, 300), dtype=torch_cuda.float64, device="cuda")
            lam, sa = api.adjoint(g, s, xi, eta, src, par, tau, rec, Rc, 1e-11, 300, kap, tile_k=tk, groups=groups,
                                  eps_hist=h, continuous=continuous, compact=compact)
            torch_cuda.cuda.synchronize()
            got = [x.cpu().numpy() for x in (lam, sa, h)]
            if ref is None:
                ref = got
                continue
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (continuous, compact, tk, groups)
            if tk == 0:
                assert np.array_equal(got[2], ref[2]), (continuous, compact, groups)
            else:
                assert np.allclose(got[2], ref[2], rtol=1e-12, atol=0.0), (continuous, compact, tk, groups)
    o = oracle_path(wl, 1e-11, 300, R=wl["R"])
    lam, sa = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, 1e-11, 300, kap, compact=True)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(sa.cpu().numpy(), o["it_a"])
    assert rel_inf(lam.cpu().numpy(), o["lam"]) <= TOL_ADJ


@pytest.mark.parametrize("zeta,eps_rel", [(0.5, 1e-3), (1.0, 0.0), (0.0, 0.1)])
def test_kernel_density_parity(torch_cuda, zeta, eps_rel):
    """Kernel-density normalisation (Eqs. (18)-(19)) through the C ABI: the
    density adjoint (every R = 1) and the data adjoint on the GPU, Kd and the
    normalised kernels against the oracle's own chain, to the adjoint
    tolerance; Kd >= 0 and, for zeta = 1 and eps = 0, the density kernel
    normalised by itself is s^2."""
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(13, 14, 15), nsrc=3, nrec=9, seed=29)
    g, kap = wl["grid"], wl["kappa"]
    s, xi, eta, src, rec, R = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "src", "rec", "R"))
    par = api.source_params(g, s, xi, eta, src)
    tau, _ = api.forward(g, s, xi, eta, src, par, 1e-13, 1000, kap, poll=True)
    lam, _ = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, 1e-13, 1000, kap, poll=True)
    grad = api.kernel(g, s, xi, eta, src, par, tau, lam)
    ones = torch_cuda.ones_like(R)
    lam1, _ = api.adjoint(g, s, xi, eta, src, par, tau, rec, ones, 1e-13, 1000, kap, poll=True)
    dens = api.kernel(g, s, xi, eta, src, par, tau, lam1)[0].contiguous()
    o = oracle_path(wl, 1e-13, 1000, R=wl["R"])
    od = np.zeros((3,) + tuple(g["n"]))
    for q in range(3):
        rhs = O.adjoint_rhs(g, wl["src"][q], o["par"][q], wl["rec"], np.ones(len(wl["rec"])))
        l1, _, conv, _ = O.adjoint(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], o["par"][q], kap, o["tau"][q], rhs,
                                   1e-13, 1000)
        assert conv
        O.kernel(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], o["par"][q], kap, o["tau"][q], l1, od)
    _, Kd_o = O.kernel_density(g, wl["s"], od[0], o["grad"], 0.0, 0.0)
    eps = eps_rel * Kd_o.max()
    K_o, Kd_o = O.kernel_density(g, wl["s"], od[0], o["grad"], eps, zeta)
    K, Kd = api.kernel_density(g, s, dens, grad, eps, zeta)
    K, Kd = K.cpu().numpy(), Kd.cpu().numpy()
    assert Kd.min() >= -1e-13 * Kd.max()
    assert rel_inf(Kd, Kd_o) <= TOL_ADJ
    fin = np.isfinite(K_o).all(axis=0)
    if eps == 0.0 and zeta > 0.0:  # K / Kd^zeta is ill-conditioned where Kd underflows towards 0
        fin &= Kd_o > 1e-8 * Kd_o.max()
    assert fin[1:-1, 1:-1, 1:-1].mean() > 0.8
    for c in range(3):
        assert rel_inf(K[c][fin], K_o[c][fin]) <= TOL_ADJ, c
    if zeta == 1.0 and eps == 0.0:
        Ks_self, _ = api.kernel_density(g, s, dens, api.kernel(g, s, xi, eta, src, par, tau, lam1), 0.0, 1.0)
        live = Kd > 1e-10 * Kd.max()
        assert np.allclose(Ks_self[0].cpu().numpy()[live], wl["s"][live] ** 2, rtol=1e-12)


def test_invalid_arguments_rejected(torch_cuda):
    from paper_2412_00031_amd import api, _lib
    wl = W.small_spherical(n=(6, 6, 6), nsrc=1)
    g = wl["grid"]
    s, xi, eta, src = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "src"))
    par = api.source_params(g, s, xi, eta, src)
    for kw in (dict(tile_k=63), dict(tile_k=-1), dict(groups=-1), dict(groups=9)):
        with pytest.raises(_lib.TTError):
            api.forward(g, s, xi, eta, src, par, 1e-6, 10, 1.05, ws=torch_cuda.empty(1 << 20, dtype=torch_cuda.uint8,
                                                                                     device="cuda"), **kw)
    with pytest.raises(_lib.TTError):
        api.forward(g, s, xi, eta, src, par, 0.0, 10, 1.05)
    with pytest.raises(_lib.TTError):
        api.forward(g, s, xi, eta, src, par, 1e-6, 0, 1.05)
    bad = dict(g, n=(3, 6, 6))
    with pytest.raises((_lib.TTError, ValueError)):
        api.forward(bad, s[:108], xi[:108], eta[:108], src, par, 1e-6, 10, 1.05)


def test_misfit_with_pairs(torch_cuda):
    from paper_2412_00031_amd import api
    rng = np.random.default_rng(5)
    nsrc, nrec, npair = 7, 40, 150
    T = rng.uniform(1, 20, (nsrc, nrec))
    Tobs = T + rng.normal(0, 0.2, T.shape)
    w = rng.uniform(0.5, 1.5, T.shape)
    pairs = W.random_pairs(nrec, npair, rng)
    wpair = rng.uniform(0.5, 2.0, (nsrc, npair))
    chi_o, R_o = O.misfit(T, Tobs, w, pairs, wpair, alpha=0.7, beta=1.3)
    chi_g, R_g = api.misfit(_dev(torch_cuda, T), _dev(torch_cuda, Tobs), _dev(torch_cuda, w),
                            _dev(torch_cuda, pairs, torch_cuda.int32), _dev(torch_cuda, wpair), 0.7, 1.3)
    assert abs(chi_g.item() - chi_o) <= 1e-13 * abs(chi_o)
    assert rel_inf(R_g.cpu().numpy(), R_o) <= 1e-14


def test_misfit_path_with_pairs_spherical(torch_cuda):
    wl = W.small_spherical(n=(12, 13, 17), nsrc=2, nrec=12, seed=21)
    rng = np.random.default_rng(22)
    wl["pairs"] = W.random_pairs(len(wl["rec"]), 20, rng)
    T_obs = W.straight_line_times(wl["grid"], wl["src"], wl["rec"], 6.3)
    op = oracle_path(wl, 1e-11, 300, T_obs=T_obs)
    gp = gpu_path(torch_cuda, wl, 1e-11, 300, T_obs=T_obs)
    # chi and R inherit the traveltime error: with |dT| <= 1e-12 max|T|,
    # |d chi| <= sum |R| |dT| and |dR_m| <= (1 + 2 * pairs touching m) |dT|
    dT = 1e-12 * np.abs(op["T"]).max()
    assert abs(gp["chi"] - op["chi"]) <= np.abs(op["R"]).sum() * dT + 1e-15 * abs(op["chi"])
    touch = np.bincount(wl["pairs"].reshape(-1), minlength=op["R"].shape[1])
    assert (np.abs(gp["R"] - op["R"]) <= (1 + 2 * touch)[None, :] * dT + 1e-15).all()
    assert_parity(gp, op)


def _cr_inputs(nsrc, nrec, per_rec, seed, empty_every=0):
    rng = np.random.default_rng(seed)
    off, pair, tri = W.receiver_source_pairs(nsrc, nrec, per_rec, rng)
    if empty_every:
        # receivers without any pair: drop every empty_every-th receiver's list
        keep = tri[:, 2] % empty_every != 0
        tri = tri[keep]
        pair = tri[:, :2].copy()
        off = np.concatenate([[0], np.cumsum(np.bincount(tri[:, 2], minlength=nrec))]).astype(np.int32)
    return dict(off=off, pair=np.ascontiguousarray(pair), tri=np.ascontiguousarray(tri),
                w=rng.uniform(0.5, 2.0, len(tri)), gamma=0.9)


@pytest.mark.parametrize("nsrc,nrec,per_rec,empty_every", [(9, 300, 12, 0), (5, 40, 10, 3), (2, 7, 1, 0)])
def test_misfit_cr_parity(torch_cuda, nsrc, nrec, per_rec, empty_every):
    """Eq. (1) with all three misfits against the oracle: chi to 1e-13, R to
    1e-14 (each R element sees the same additions in the same order; only
    contraction of multiply-adds differs).  300 receivers exceed one pass of the
    256-thread block; receivers with no pair and a single pair per receiver are
    covered."""
    from paper_2412_00031_amd import api
    rng = np.random.default_rng(31 + nsrc)
    T = rng.uniform(1, 20, (nsrc, nrec))
    Tobs = T + rng.normal(0, 0.2, T.shape)
    w = rng.uniform(0.5, 1.5, T.shape)
    pairs = W.random_pairs(nrec, min(60, nrec * (nrec - 1) // 2), rng)
    cr = _cr_inputs(nsrc, nrec, per_rec, 40 + nsrc, empty_every)
    chi_o, R_o = O.misfit(T, Tobs, w, pairs, None, alpha=0.7, beta=1.3)
    chi_cr, R_o = O.misfit_cr(T, Tobs, cr["tri"], cr["w"], cr["gamma"], R_o)
    chi_o += chi_cr
    d = lambda a, dt=None: _dev(torch_cuda, a, dt)
    chi_g, R_g = api.misfit(d(T), d(Tobs), d(w), d(pairs, torch_cuda.int32), None, 0.7, 1.3,
                            cr=(d(cr["off"], torch_cuda.int32), d(cr["pair"], torch_cuda.int32)), wcr=d(cr["w"]),
                            gamma=cr["gamma"])
    assert abs(chi_g.item() - chi_o) <= 1e-13 * abs(chi_o)
    assert rel_inf(R_g.cpu().numpy(), R_o) <= 1e-14


def test_misfit_cr_no_pairs_and_bad_indices(torch_cuda):
    """No pairs (NULL pair list) leaves chi and R as tt_misfit left them; an
    out-of-range source index or a decreasing offset is skipped by the
    kernel's own checks and reported as chi = NaN."""
    from paper_2412_00031_amd import api
    rng = np.random.default_rng(50)
    T = rng.uniform(1, 20, (3, 5))
    Tobs = T + rng.normal(0, 0.2, T.shape)
    d = lambda a, dt=None: _dev(torch_cuda, a, dt)
    chi0, R0 = api.misfit(d(T), d(Tobs))
    empty = (d(np.zeros(6, np.int32), torch_cuda.int32), d(np.zeros((0, 2), np.int32), torch_cuda.int32))
    chi1, R1 = api.misfit(d(T), d(Tobs), cr=empty, gamma=2.0)
    assert chi1.item() == chi0.item() and torch_cuda.equal(R1, R0)
    bad_src = (d(np.array([0, 1, 1, 1, 1, 1], np.int32), torch_cuda.int32), d(np.array([[0, 3]], np.int32), torch_cuda.int32))
    chi2, _ = api.misfit(d(T), d(Tobs), cr=bad_src)
    assert np.isnan(chi2.item())
    bad_off = (d(np.array([0, 1, 0, 1, 1, 1], np.int32), torch_cuda.int32), d(np.array([[0, 2]], np.int32), torch_cuda.int32))
    chi3, _ = api.misfit(d(T), d(Tobs), cr=bad_off)
    assert np.isnan(chi3.item())
    bad_pair = d(np.array([[0, 7]], np.int32), torch_cuda.int32)
    chi4, _ = api.misfit(d(T), d(Tobs), pairs=bad_pair)
    assert np.isnan(chi4.item())


def test_misfit_path_with_cr_pairs_spherical(torch_cuda):
    """Forward, sampling, all three misfits, adjoint and kernels with the
    common-receiver term coupling the sources."""
    wl = W.small_spherical(n=(12, 13, 17), nsrc=4, nrec=12, seed=23)
    rng = np.random.default_rng(24)
    wl["pairs"] = W.random_pairs(len(wl["rec"]), 10, rng)
    wl["cr"] = _cr_inputs(4, len(wl["rec"]), 3, 25)
    T_obs = W.straight_line_times(wl["grid"], wl["src"], wl["rec"], 6.3)
    op = oracle_path(wl, 1e-11, 300, T_obs=T_obs)
    gp = gpu_path(torch_cuda, wl, 1e-11, 300, T_obs=T_obs)
    # chi and R inherit the traveltime error |dT| <= 1e-12 max|T|: each R
    # element moves by at most (1 + 2 * pairs touching it) |dT| times the
    # largest weight
    dT = 1e-12 * np.abs(op["T"]).max()
    assert abs(gp["chi"] - op["chi"]) <= np.abs(op["R"]).sum() * dT + 1e-15 * abs(op["chi"])
    touch = np.zeros(op["R"].shape)
    touch += np.bincount(wl["pairs"].reshape(-1), minlength=op["R"].shape[1])[None, :]
    for n, j, m in wl["cr"]["tri"]:
        touch[n, m] += 1
        touch[j, m] += 1
    wmax = max(1.0, wl["cr"]["gamma"] * wl["cr"]["w"].max())
    assert (np.abs(gp["R"] - op["R"]) <= (1 + 2 * touch) * wmax * dT + 1e-15).all()
    assert_parity(gp, op)


def test_truncated_iterations_report_nonconvergence(torch_cuda):
    wl = W.small_spherical(n=(16, 15, 14), nsrc=2, seed=3)
    op = oracle_path(wl, 1e-14, 3, R=wl["R"], max_iter_adj=2)
    gp = gpu_path(torch_cuda, wl, 1e-14, 3, R=wl["R"], max_iter_adj=2)
    assert list(op["it_f"]) == [-3, -3] and list(op["it_a"]) == [-2, -2]
    assert_parity(gp, op)


def test_warm_start_parity(torch_cuda):
    wl = W.small_spherical(n=(14, 14, 14), nsrc=2, seed=9)
    rng = np.random.default_rng(10)
    tau0 = 1.0 + 0.02 * rng.standard_normal((2,) + tuple(wl["grid"]["n"]))
    op = oracle_path(wl, 1e-11, 300, R=wl["R"], tau_init=tau0)
    gp = gpu_path(torch_cuda, wl, 1e-11, 300, R=wl["R"], tau_init=tau0)
    assert_parity(gp, op)


def test_fixed_cell_touching_boundary_and_on_node(torch_cuda):
    wl = W.small_spherical(n=(10, 11, 12), nsrc=3, seed=4)
    g = wl["grid"]
    ax = W.axes(g)
    src = wl["src"].copy()
    src[0] = [ax[0][-1] - 0.3 * g["h"][0], ax[1][0] + 0.2 * g["h"][1], ax[2][5]]      # cell at the surface/corner
    src[1] = [ax[0][4], ax[1][6], ax[2][7]]                                            # exactly on a node
    src[2] = [ax[0][0] + 0.5 * g["h"][0], ax[1][-1] - 0.1 * g["h"][1], ax[2][-1]]     # far corner
    wl["src"] = src
    op = oracle_path(wl, 1e-11, 300, R=wl["R"])
    gp = gpu_path(torch_cuda, wl, 1e-11, 300, R=wl["R"])
    assert_parity(gp, op)


def test_minimal_grid_and_cartesian_anisotropic(torch_cuda):
    rng = np.random.default_rng(8)
    for n in ((4, 4, 4), (4, 6, 5), (9, 4, 7)):
        g = W.cartesian_grid(1, 1.0)
        g["n"] = n
        s = 1.0 / rng.uniform(5.0, 7.0, n)
        xi = rng.uniform(-0.05, 0.05, n)
        eta = rng.uniform(-0.05, 0.05, n)
        L = [(v - 1) * 1.0 for v in n]
        src = np.array([[rng.uniform(0, L[0]), rng.uniform(0, L[1]), rng.uniform(0, L[2])]])
        rec = np.array([[0.0, rng.uniform(0, L[1]), rng.uniform(0, L[2])] for _ in range(3)])
        wl = dict(grid=g, s=s, xi=xi, eta=eta, src=src, rec=rec, R=rng.normal(0, 0.1, (1, 3)), kappa=1.12)
        op = oracle_path(wl, 1e-12, 300, R=wl["R"])
        gp = gpu_path(torch_cuda, wl, 1e-12, 300, R=wl["R"])
        assert_parity(gp, op)


def test_empty_batch_is_a_no_op(torch_cuda):
    """Zero sources through every step of the path: the solves and sampling
    return empty results, chi is zero, and the kernels write zeros (or leave an
    accumulated gradient unchanged)."""
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(9, 10, 11), nsrc=1, nrec=4, seed=3)
    g = wl["grid"]
    s, xi, eta, rec = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "rec"))
    src = torch_cuda.zeros((0, 3), dtype=torch_cuda.float64, device="cuda")
    par = api.source_params(g, s, xi, eta, src)
    tau, st = api.forward(g, s, xi, eta, src, par, 1e-8, 50, wl["kappa"])
    assert tau.shape == (0,) + tuple(g["n"]) and st.numel() == 0
    T = api.sample(g, src, par, tau, rec)
    assert T.shape == (0, len(wl["rec"]))
    chi, R = api.misfit(T, T.clone())
    assert chi.item() == 0.0 and R.numel() == 0
    lam, st = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, 1e-8, 50, wl["kappa"])
    assert lam.shape == tau.shape and st.numel() == 0
    grad = api.kernel(g, s, xi, eta, src, par, tau, lam)
    assert torch_cuda.count_nonzero(grad).item() == 0
    prior = torch_cuda.full_like(grad, 0.25)
    assert torch_cuda.equal(api.kernel(g, s, xi, eta, src, par, tau, lam, grad=prior.clone()), prior)


def test_maximum_source_count(torch_cuda):
    """The largest batch the entry points take (65535 sources: one launch
    dimension per source) on a minimal spherical grid: forward, sampling and
    adjoint over the whole batch, checked against the oracle on sampled sources
    (both ends, and both sides of every boundary between the 4 source groups),
    iteration counts included; 65536 sources are refused."""
    from paper_2412_00031_amd import api, _lib
    wl = W.small_spherical(n=(5, 6, 7), nsrc=1, nrec=6, seed=31)
    g, kap = wl["grid"], wl["kappa"]
    rng = np.random.default_rng(32)
    nmax = 65535
    lo, span = np.array(g["o"], float), (np.array(g["n"]) - 1) * np.array(g["h"], float)
    src = lo + rng.uniform(0.05, 0.95, (nmax, 3)) * span
    R = rng.normal(0.0, 0.1, (nmax, len(wl["rec"])))
    s, xi, eta, rec = (_dev(torch_cuda, wl[k]) for k in ("s", "xi", "eta", "rec"))
    srcd = _dev(torch_cuda, src)
    par = api.source_params(g, s, xi, eta, srcd)
    tau, st_f = api.forward(g, s, xi, eta, srcd, par, 1e-11, 300, kap, poll=True)
    T = api.sample(g, srcd, par, tau, rec)
    lam, st_a = api.adjoint(g, s, xi, eta, srcd, par, tau, rec, _dev(torch_cuda, R), 1e-11, 300, kap, poll=True)
    torch_cuda.cuda.synchronize()
    sel = [0, 1, 16383, 16384, 32767, 32768, 49151, 49152, nmax - 1]
    par_o = O.source_params(g, wl["s"], wl["xi"], wl["eta"], src[sel])
    assert rel_inf(par[sel].cpu().numpy(), par_o) <= 1e-15
    for n, q in enumerate(sel):
        tau_o, it, conv, _ = O.forward(g, wl["s"], wl["xi"], wl["eta"], src[q], par_o[n], kap, 1e-11, 300)
        assert int(st_f[q]) == (it if conv else -it), q
        assert rel_inf(tau[q].cpu().numpy(), tau_o) <= TOL_TAU, q
        T_o = O.sample(g, src[q], par_o[n], tau_o, wl["rec"])
        assert rel_inf(T[q].cpu().numpy(), T_o) <= TOL_TAU, q
        rhs = O.adjoint_rhs(g, src[q], par_o[n], wl["rec"], R[q])
        lam_o, it, conv, _ = O.adjoint(g, wl["s"], wl["xi"], wl["eta"], src[q], par_o[n], kap, tau_o, rhs, 1e-11,
                                       300)
        assert int(st_a[q]) == (it if conv else -it), q
        assert rel_inf(lam[q].cpu().numpy(), lam_o) <= TOL_ADJ, q
    assert (st_f > 0).all() and (st_a > 0).all()
    del lam, tau
    one = _dev(torch_cuda, np.concatenate([src, src[:1]]))
    with pytest.raises(_lib.TTError):
        api.forward(g, s, xi, eta, one, torch_cuda.cat([par, par[:1]]), 1e-11, 300, kap)


@pytest.mark.slow
def test_sph61_all_sources_summed_kernels(torch_cuda):
    """The 61^3 spherical workload with all of its 32 sources: iteration
    counts, fields of every source and the kernels summed over all 32
    (Eqs. (6)-(8)) against the oracle (its sources solved on parallel host
    threads, summed in ascending source order)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    wl = W.sph61(nsrc=32)
    g, kap, tol = wl["grid"], wl["kappa"], wl["tol"]
    gp = gpu_path(torch_cuda, wl, tol, 300, R=wl["R"])
    par = O.source_params(g, wl["s"], wl["xi"], wl["eta"], wl["src"])

    def solve(q):
        tau, itf, cf, _ = O.forward(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], par[q], kap, tol, 300)
        rhs = O.adjoint_rhs(g, wl["src"][q], par[q], wl["rec"], wl["R"][q])
        lam, ita, ca, _ = O.adjoint(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], par[q], kap, tau, rhs, tol, 300)
        return tau, (itf if cf else -itf), lam, (ita if ca else -ita)

    with ThreadPoolExecutor(max(1, min(16, len(os.sched_getaffinity(0))))) as ex:
        res = list(ex.map(solve, range(32)))
    grad = np.zeros((3,) + tuple(g["n"]))
    for q, (tau, itf, lam, ita) in enumerate(res):
        assert itf == gp["it_f"][q] and ita == gp["it_a"][q], q
        assert rel_inf(gp["tau"][q], tau) <= TOL_TAU, q
        assert rel_inf(gp["lam"][q], lam) <= TOL_ADJ, q
        O.kernel(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], par[q], kap, tau, lam, grad)
    assert (gp["it_f"] > 0).all() and (gp["it_a"] > 0).all()
    for c in range(3):
        assert rel_inf(gp["grad"][c], grad[c]) <= TOL_ADJ, (c, rel_inf(gp["grad"][c], grad[c]))
