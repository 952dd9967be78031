"""Pins of the FP64 NumPy U-Net reference: layers against brute-force loops
written from their definitions, the whole backward pass against central finite
differences, and Adam's first step against its closed form."""
import numpy as np

from oracle import unet_ref as U


def _conv_loops(x, W, b):
    D, H, Wd, C = x.shape
    y = np.zeros((D, H, Wd, W.shape[2]))
    for z in range(D):
        for yy in range(H):
            for xx in range(Wd):
                acc = b.copy()
                for t, (dz, dy, dx) in enumerate(U._TAPS):
                    q = (z + dz, yy + dy, xx + dx)
                    if all(0 <= q[a] < (D, H, Wd)[a] for a in range(3)):
                        acc = acc + x[q] @ W[t]
                y[z, yy, xx] = acc
    return y


def test_layers_against_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4, 5, 6, 3))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    assert np.allclose(U.conv3(x, W, b), _conv_loops(x, W, b), rtol=1e-13, atol=1e-13)
    xe = rng.standard_normal((4, 6, 2, 3))
    p = U.pool(xe)
    for z in range(2):
        for yy in range(3):
            for xx in range(1):
                assert np.array_equal(p[z, yy, xx], xe[2 * z:2 * z + 2, 2 * yy:2 * yy + 2, 2 * xx:2 * xx + 2].max(axis=(0, 1, 2)))
    Wu = rng.standard_normal((8, 3, 2))
    yu = U.up(xe, Wu, b)
    for s, (a, bb, c) in enumerate(U._SUB):
        assert np.allclose(yu[1 * 2 + a, 3 * 2 + bb, 1 * 2 + c], xe[1, 3, 1] @ Wu[s] + b)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    P = U.init_params(rng, ch=(2, 3, 3, 4))
    for k in P:
        if k.endswith(".b"):
            P[k] = 0.1 * rng.standard_normal(P[k].shape)
    x = rng.standard_normal((8, 8, 8, U.IN_CH))
    gy = rng.standard_normal((8, 8, 8))
    y, cache = U.forward(P, x)
    G = U.backward(P, cache, gy)
    L = lambda Q: float((U.forward(Q, x)[0] * gy).sum())
    h = 1e-6
    checked = 0
    for name in sorted(P):
        flat = P[name].reshape(-1)
        for idx in rng.choice(flat.size, min(3, flat.size), replace=False):
            Qp = {k: v.copy() for k, v in P.items()}
            Qm = {k: v.copy() for k, v in P.items()}
            Qp[name].reshape(-1)[idx] += h
            Qm[name].reshape(-1)[idx] -= h
            fd = (L(Qp) - L(Qm)) / (2 * h)
            an = G[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)
            checked += 1
    assert checked > 40


def test_mse_and_adam_first_step():
    rng = np.random.default_rng(2)
    y, t = rng.standard_normal((4, 4, 4)), rng.standard_normal((4, 4, 4))
    mask = rng.random((4, 4, 4)) > 0.3
    loss, g = U.mse(y, t, mask)
    assert abs(loss - ((y - t)[mask] ** 2).mean()) < 1e-14
    e = 1e-7
    y2 = y.copy(); y2[1, 2, 3] += e
    assert abs((U.mse(y2, t, mask)[0] - loss) / e - g[1, 2, 3]) < 1e-5
    w = rng.random((4, 4, 4))  # fractional weights
    lw, gw = U.mse(y, t, w)
    assert abs(lw - (w * (y - t) ** 2).sum() / w.sum()) < 1e-14
    y2 = y.copy(); y2[2, 0, 1] += e
    assert abs((U.mse(y2, t, w)[0] - lw) / e - gw[2, 0, 1]) < 1e-5
    p, gg = rng.standard_normal(5), rng.standard_normal(5)
    p1, m1, v1 = U.adam(p, gg, np.zeros(5), np.zeros(5), 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * gg / (np.abs(gg) + 1e-8), rtol=1e-12, atol=1e-15)
