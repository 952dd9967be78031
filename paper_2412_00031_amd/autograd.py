"""Differentiable traveltime misfit: chi(s, xi, eta) as a torch.autograd.Function.

Forward: batched fast-sweeping solve (Sec. 2.1 step 1), receiver traveltimes
and the misfit chi = alpha chi_t + beta chi_cs + gamma chi_cr (Eqs. (1)-(4)).
Backward: the adjoint solve at the adjoint sources R = d chi / d T (Eq. (5),
(A2)-(A4)) and
the kernels (Eqs. (6)-(8)) scaled by the incoming gradient.  Both passes run
in libtt through the C ABI; this module only routes tensors.

The source constants s0, xi0, eta0 of the factorisation are not
differentiated: pass them in ``problem["src_par"]`` to hold them fixed (for
finite-difference checks), or let the forward take them from the model.
"""
import torch

from . import api


class NotConverged(RuntimeError):
    """A solve of the misfit or its gradient reached max_iter before tol."""


def _check_status(status, what):
    bad = (status <= 0).nonzero().flatten().tolist()
    if bad:
        its = (-status[bad]).tolist()
        raise NotConverged(f"{what} solve did not converge for source(s) {bad[:16]}{' ...' if len(bad) > 16 else ''} "
                           f"within max_iter ({its[:16]} iterations); raise max_iter or tol")


class EikonalMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, xi, eta, problem):
        g = problem["grid"]
        src, rec, T_obs = problem["src"], problem["rec"], problem["T_obs"]
        tol, max_iter, kappa = problem["tol"], problem.get("max_iter", 2000), problem["kappa"]
        par = problem.get("src_par")
        if par is None:
            par = api.source_params(g, s.detach(), xi.detach(), eta.detach(), src)
        tau, st = api.forward(g, s.detach(), xi.detach(), eta.detach(), src, par, tol, max_iter, kappa,
                              tile_k=problem.get("tile_k_fwd", 0), poll=True)
        _check_status(st, "forward")
        T = api.sample(g, src, par, tau, rec)
        chi, R = api.misfit(T, T_obs, problem.get("w"), problem.get("pairs"), problem.get("wpair"),
                            problem.get("alpha", 1.0), problem.get("beta", 1.0), problem.get("cr"),
                            problem.get("wcr"), problem.get("gamma", 1.0))
        ctx.save_for_backward(s.detach(), xi.detach(), eta.detach(), tau, R, par)
        ctx.problem = problem
        return chi

    @staticmethod
    def backward(ctx, grad_chi):
        s, xi, eta, tau, R, par = ctx.saved_tensors
        p = ctx.problem
        g = p["grid"]
        lam, st = api.adjoint(g, s, xi, eta, p["src"], par, tau, p["rec"], R, p.get("adj_tol", p["tol"]),
                              p.get("adj_max_iter", p.get("max_iter", 2000)), p["kappa"],
                              tile_k=p.get("tile_k_adj", 0),
                              continuous=p.get("continuous_adjoint", False), poll=True)
        _check_status(st, "adjoint")
        grad = api.kernel(g, s, xi, eta, p["src"], par, tau, lam)
        grad = grad * grad_chi.to(grad.dtype)
        return grad[0], grad[1], grad[2], None


def misfit(s, xi, eta, problem):
    """chi(s, xi, eta) for the sources, receivers and observations in
    ``problem`` (keys: grid, src, rec, T_obs, tol, kappa, optional max_iter,
    adj_tol, adj_max_iter, src_par, w, pairs, wpair, alpha, beta, cr = (cr_off, cr_pair), wcr,
    gamma, tile_k_fwd, tile_k_adj, continuous_adjoint; see api.misfit).  With
    continuous_adjoint the backward takes the upwind solution of Eq. (5): the
    paper's gradient, first-order close to the exact derivative.  Both solves
    are host-polled and raise NotConverged, naming the sources, when a source
    reaches max_iter before tol (chi and its gradient are defined by converged
    fields)."""
    return EikonalMisfit.apply(s, xi, eta, problem)
