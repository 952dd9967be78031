"""The whole per-source step captured into a caller's hipGraph.

Source constants, forward solve, receiver traveltimes, misfit and adjoint
sources (Eqs. (2), (A2)), adjoint solve and kernels (Eqs. (6)-(8)) are
enqueued through the C ABI on a stream that torch is capturing; the graph is
replayed several times, with eager work and synchronisations in between, and
every replay must equal the eager step bit for bit (and the oracle to the
parity tolerances).  The solves run asynchronously: max_iter is the iteration
budget, converged sources exit on the device, and nothing waits on the host.
"""
import numpy as np
import pytest

import oracle as O
from conftest import rel_inf
from paper_2412_00031_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


@pytest.mark.parametrize("groups", [1, 2])
def test_captured_step_matches_eager_and_oracle(torch_cuda, groups):
    torch = torch_cuda
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(14, 13, 15), nsrc=4, nrec=8, seed=41)
    g, kap, tol, budget = wl["grid"], wl["kappa"], 1e-10, 120
    s, xi, eta, src, rec = (_dev(torch, wl[k]) for k in ("s", "xi", "eta", "src", "rec"))
    T_obs = _dev(torch, W.straight_line_times(g, wl["src"], wl["rec"], 6.2))

    def step():
        par = api.source_params(g, s, xi, eta, src)
        tau, st_f = api.forward(g, s, xi, eta, src, par, tol, budget, kap, groups=groups)
        T = api.sample(g, src, par, tau, rec)
        chi, R = api.misfit(T, T_obs)
        lam, st_a = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, tol, budget, kap, groups=groups)
        grad = api.kernel(g, s, xi, eta, src, par, tau, lam)
        return dict(par=par, tau=tau, st_f=st_f, T=T, chi=chi, R=R, lam=lam, st_a=st_a, grad=grad)

    # eager reference (also creates the library's helper streams and events
    # before the capture)
    ref = step()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    assert (ref["st_f"] > 0).all() and (ref["st_a"] > 0).all()

    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                                  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        out = step()
    for rep in range(3):
        for v in out.values():
            v.fill_(-7.0) if v.dtype == torch.float64 else v.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (rep, k)
        _ = (out["tau"] * 3.0).sum().item()     # eager work between replays
        torch.cuda.synchronize()

    # the replayed results are the oracle's (iteration counts included)
    r = {k: v.cpu().numpy() for k, v in out.items()}
    par_o = O.source_params(g, wl["s"], wl["xi"], wl["eta"], wl["src"])
    grad_o = np.zeros((3,) + tuple(g["n"]))
    taus = []
    for q in range(len(wl["src"])):
        tau_o, it, conv, _ = O.forward(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], par_o[q], kap, tol, budget)
        assert conv and it == r["st_f"][q]
        assert rel_inf(r["tau"][q], tau_o) <= 1e-12
        taus.append(tau_o)
    T_o = np.stack([O.sample(g, wl["src"][q], par_o[q], taus[q], wl["rec"]) for q in range(len(taus))])
    assert rel_inf(r["T"], T_o) <= 1e-12
    chi_o, R_o = O.misfit(T_o, T_obs.cpu().numpy())
    assert abs(float(r["chi"]) - chi_o) <= 1e-10 * abs(chi_o)
    for q in range(len(taus)):
        rhs = O.adjoint_rhs(g, wl["src"][q], par_o[q], wl["rec"], R_o[q])
        lam_o, it, conv, _ = O.adjoint(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], par_o[q], kap, taus[q], rhs,
                                       tol, budget)
        assert conv and it == r["st_a"][q]
        assert rel_inf(r["lam"][q], lam_o) <= 1e-10
        O.kernel(g, wl["s"], wl["xi"], wl["eta"], wl["src"][q], par_o[q], kap, taus[q], lam_o, grad_o)
    for c in range(3):
        assert rel_inf(r["grad"][c], grad_o[c]) <= 1e-10, c


def test_budget_exhausted_reports_no_convergence(torch_cuda):
    """An asynchronous solve whose budget is too small for a source reports
    -iterations for it (the no-convergence condition) and still writes its
    field; the polled solve with the same budget gives the same numbers."""
    torch = torch_cuda
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(12, 13, 11), nsrc=3, nrec=5, seed=43)
    g, kap = wl["grid"], wl["kappa"]
    s, xi, eta, src = (_dev(torch, wl[k]) for k in ("s", "xi", "eta", "src"))
    par = api.source_params(g, s, xi, eta, src)
    tau_a, st_a = api.forward(g, s, xi, eta, src, par, 1e-12, 3, kap)
    tau_p, st_p = api.forward(g, s, xi, eta, src, par, 1e-12, 3, kap, poll=True)
    torch.cuda.synchronize()
    assert (st_a.cpu().numpy() == -3).all() and torch.equal(st_a, st_p) and torch.equal(tau_a, tau_p)
