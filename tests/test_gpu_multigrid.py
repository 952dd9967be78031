"""Multiple-grid parameterisation (Eqs. (11)-(17)) on the GPU against the
oracle: projection of kernels onto the inversion-grid basis and expansion of
coefficients into fields, on a small spherical grid and on the 101^3 grid."""
import numpy as np
import pytest

import oracle as O
from conftest import rel_inf
from paper_2412_00031_amd import workloads as W

pytestmark = pytest.mark.gpu


def _inv_grids(g, seed, sizes=((4, 3, 5), (5, 4, 4))):
    """Staggered inversion grids with uneven spacing and margins past the
    forward grid's ends (the second one offset further)."""
    rng = np.random.default_rng(seed)
    ax = W.axes(g)
    grids = []
    for q, m in enumerate(sizes):
        axes = []
        for a in range(3):
            lo, hi = ax[a][0], ax[a][-1]
            span = hi - lo
            c = np.sort(lo + span * np.concatenate([[-0.05 - 0.1 * q], rng.uniform(0.1, 0.9, m[a] - 2),
                                                     [1.05 + 0.1 * q]]))
            axes.append(c)
        grids.append(tuple(axes))
    return grids


@pytest.mark.parametrize("case", ["small", "sph101", "sph101_staggered5", "wave_per_node"])
def test_multigrid_project_expand_parity(torch_cuda, case):
    from paper_2412_00031_amd import api
    torch = torch_cuda
    if case == "small":
        g = W.small_spherical(n=(13, 14, 15), seed=3)["grid"]
        inv = _inv_grids(g, 7)
    elif case == "sph101":
        g = W.spherical_grid(101, 100.0, 2.0)
        inv = _inv_grids(g, 11, sizes=((11, 13, 12), (12, 11, 13)))
    elif case == "wave_per_node":
        # inversion grids whose staged form does not fit in LDS: one wave per node
        g = W.small_spherical(n=(13, 14, 15), seed=3)["grid"]
        inv = _inv_grids(g, 9, sizes=((5, 70, 70), (4, 66, 71)))
        assert api.mg_workspace_size(g, inv) == 0
    else:
        # the inversion grids that the benchmark times: 5 staggered 11 x 13 x 13 grids
        g = W.spherical_grid(101, 100.0, 2.0)
        inv = W.staggered_inversion_grids(g, (11, 13, 13), 5)
    rng = np.random.default_rng(5)
    K = rng.standard_normal((3,) + tuple(g["n"]))
    P_o = O.mg_project(g, inv, K)
    P = api.mg_project(g, inv, torch.as_tensor(K, device="cuda"))
    for p_o, p in zip(P_o, P):
        assert rel_inf(p.cpu().numpy(), p_o) <= 1e-12
    C = [rng.standard_normal((3,) + tuple(len(c) for c in axes)) for axes in inv]
    F_o = O.mg_expand(g, inv, C)
    F = api.mg_expand(g, inv, [torch.as_tensor(c, device="cuda") for c in C]).cpu().numpy()
    assert rel_inf(F, F_o) <= 1e-13
    # the projection is the transpose of the expansion under the node quadrature (on the GPU alone)
    V = O.node_volume(g)
    lhs = sum(float((p.cpu().numpy() * c).sum()) for p, c in zip(P, C))
    rhs = float((K * V[None] * F).sum())
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + abs(rhs))


def test_multigrid_rejects_bad_sizes(torch_cuda):
    from paper_2412_00031_amd import _lib, api
    torch = torch_cuda
    g = W.small_spherical(n=(6, 6, 6), seed=3)["grid"]
    K = torch.zeros((3, 6, 6, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.TTError):
        api.mg_project(g, [(np.zeros(0), np.zeros(2), np.zeros(2))], K)
