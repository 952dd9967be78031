"""Adjoint solve started from a given field (TT_FLAG_ADJOINT_INIT).

The start changes only where the Gauss-Seidel iteration begins: from zeros it
is the plain solve bit for bit, from the converged field it stops after at
most two iterations, and from a perturbed field it converges to the same
fixed point within what the tolerance allows (checked against a solve to
1e-14).  The plain solve itself is held to the oracle by the parity tests."""
import numpy as np
import pytest

from paper_2412_00031_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_adjoint_from_initial_field(torch_cuda):
    torch = torch_cuda
    from paper_2412_00031_amd import api
    wl = W.small_spherical(n=(14, 15, 16), nsrc=3, seed=21)
    g, kap = wl["grid"], wl["kappa"]
    s, xi, eta, src, rec, R = (_dev(torch, wl[k]) for k in ("s", "xi", "eta", "src", "rec", "R"))
    par = api.source_params(g, s, xi, eta, src)
    tau, st_f = api.forward(g, s, xi, eta, src, par, 1e-12, 500, kap, poll=True)
    tol = 1e-9

    def solve(init, tol_=tol, tile_k=0):
        out = torch.empty_like(tau)
        lam, st = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, tol_, 500, kap, poll=True, lam_init=init,
                              out=out, tile_k=tile_k)
        torch.cuda.synchronize()
        return lam.clone(), st.cpu().numpy()

    lam0, it0 = solve(None)
    assert (it0 > 0).all()
    # zeros: the plain solve, bit for bit
    lz, itz = solve(torch.zeros_like(tau))
    assert np.array_equal(itz, it0) and torch.equal(lz, lam0)
    # the converged field, passed as the output tensor itself (in place)
    lc = lam0.clone()
    lam1, st1 = api.adjoint(g, s, xi, eta, src, par, tau, rec, R, tol, 500, kap, poll=True, lam_init=lc, out=lc)
    torch.cuda.synchronize()
    it1 = st1.cpu().numpy()
    assert ((it1 >= 1) & (it1 <= 2)).all(), it1
    ref, itr = solve(None, 1e-14)
    assert (itr > 0).all()
    scale = ref.abs().amax(dim=(1, 2, 3))
    err = lambda a: ((a - ref).abs().amax(dim=(1, 2, 3)) / scale).cpu().numpy()
    e0 = err(lam0)
    assert (err(lam1) <= e0 + 1e-12).all()
    # a perturbed start (fixed-cell nodes are reset to 0 by the solve) at
    # another tile depth: same fixed point within the tolerance's reach
    rng = np.random.default_rng(22)
    pert = lam0 * (1.0 + 0.3 * _dev(torch, rng.standard_normal(tuple(lam0.shape))))
    lp, itp = solve(pert, tile_k=5)
    assert (itp > 0).all()
    assert (err(lp) <= np.maximum(10 * e0, 1e-7)).all(), (err(lp), e0)
