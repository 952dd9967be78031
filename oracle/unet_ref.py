"""FP64 NumPy reference of the warm-start 3-D U-Net (test infrastructure only).

Written directly from the definitions of the layers, with no blocking:
  conv3(x, W, b)[p, o] = b[o] + sum_{t in 3^3} sum_i x[p + d_t, i] W[t, i, o]   (zero padding 1)
  pool(x)[p, c]        = max over the 2^3 children of p
  up(x, W, b)[2p + a, o] = b[o] + sum_i x[p, i] W[a, i, o]                   (a in 2^3)
  head(x, w, b)[p]     = b + sum_i x[p, i] w[i]
  relu, mean-squared error, and Adam.
Activations are [D, H, W, C] (channels last); tap t = (dz+1)*9 + (dy+1)*3 + (dx+1).
Architecture: channels (16, 32, 32, 64), 4 input features, 1 output; two 3^3
convolutions with ReLU per level, 2^3 max pooling down, 2^3 stride-2 transposed
convolutions up, skip concatenation [up, skip], 1x1 head.
"""
import numpy as np

CH = (16, 32, 32, 64)
IN_CH = 4

_TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
_SUB = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]


def conv3(x, W, b):
    D, H, Wd, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (D, H, Wd, W.shape[2])).astype(np.float64).copy()
    for t, (dz, dy, dx) in enumerate(_TAPS):
        y += xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd, :] @ W[t]
    return y


def conv3_backward(x, W, gy):
    """Gradients of sum(gy * conv3(x, W, b)) with respect to x, W, b."""
    D, H, Wd, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(_TAPS):
        sl = (slice(1 + dz, 1 + dz + D), slice(1 + dy, 1 + dy + H), slice(1 + dx, 1 + dx + Wd))
        gW[t] = np.einsum("zyxi,zyxo->io", xp[sl], gy)
        gxp[sl] += gy @ W[t].T
    return gxp[1:-1, 1:-1, 1:-1, :], gW, gy.sum(axis=(0, 1, 2))


def pool(x):
    D, H, Wd, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, Wd // 2, 2, C).max(axis=(1, 3, 5))


def pool_backward(x, gy):
    """Gradient routed to the first maximum of each 2^3 block (z, y, x order)."""
    D, H, Wd, C = x.shape
    gx = np.zeros_like(x)
    blocks = x.reshape(D // 2, 2, H // 2, 2, Wd // 2, 2, C).transpose(0, 2, 4, 1, 3, 5, 6).reshape(
        D // 2, H // 2, Wd // 2, 8, C)
    arg = blocks.argmax(axis=3)
    for s, (a, b_, c) in enumerate(_SUB):
        gx[a::2, b_::2, c::2, :] = np.where(arg == s, gy, 0.0)
    return gx


def up(x, W, b):
    D, H, Wd, _ = x.shape
    y = np.zeros((2 * D, 2 * H, 2 * Wd, W.shape[2]))
    for s, (a, b_, c) in enumerate(_SUB):
        y[a::2, b_::2, c::2, :] = x @ W[s] + b
    return y


def up_backward(x, W, gy):
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for s, (a, b_, c) in enumerate(_SUB):
        g = gy[a::2, b_::2, c::2, :]
        gx += g @ W[s].T
        gW[s] = np.einsum("zyxi,zyxo->io", x, g)
    return gx, gW, gy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def init_params(rng, ch=CH, in_ch=IN_CH):
    """He-normal initialisation; returns a dict of float64 arrays."""
    c1, c2, c3, c4 = ch
    convs = [("e1a", in_ch, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2), ("e3a", c2, c3),
             ("e3b", c3, c3), ("bna", c3, c4), ("bnb", c4, c4), ("d3a", 2 * c3, c3), ("d3b", c3, c3),
             ("d2a", 2 * c2, c2), ("d2b", c2, c2), ("d1a", 2 * c1, c1), ("d1b", c1, c1)]
    ups = [("u3", c4, c3), ("u2", c3, c2), ("u1", c2, c1)]
    P = {}
    for name, ci, co in convs:
        P[name + ".W"] = rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci))
        P[name + ".b"] = np.zeros(co)
    for name, ci, co in ups:
        P[name + ".W"] = rng.standard_normal((8, ci, co)) * np.sqrt(2.0 / ci)
        P[name + ".b"] = np.zeros(co)
    P["head.W"] = rng.standard_normal((c1, 1)) * np.sqrt(1.0 / c1)
    P["head.b"] = np.zeros(1)
    return P


def _ident(a):
    return a


def forward(P, x, q=None):
    """x [D, H, W, IN_CH] (D, H, W multiples of 8) -> (y [D, H, W], cache).

    q (default: identity) is applied to the 3^3 convolution weights and to every
    stored activation (each convolution's ReLU output and each up-sampling's
    output); passing a rounding function evaluates the same network with those
    tensors held in a narrower storage format, the rest in float64."""
    q = q or _ident
    c = {}
    def cr(name, inp):
        c[name + ".in"] = inp
        z = conv3(inp, q(P[name + ".W"]), P[name + ".b"])
        c[name + ".z"] = z
        return q(relu(z))
    e1 = cr("e1b", cr("e1a", x))
    p1 = pool(e1); c["p1.in"] = e1
    e2 = cr("e2b", cr("e2a", p1))
    p2 = pool(e2); c["p2.in"] = e2
    e3 = cr("e3b", cr("e3a", p2))
    p3 = pool(e3); c["p3.in"] = e3
    bn = cr("bnb", cr("bna", p3))
    c["u3.in"] = bn
    u3 = q(up(bn, P["u3.W"], P["u3.b"]))
    d3 = cr("d3b", cr("d3a", np.concatenate([u3, e3], axis=3)))
    c["u2.in"] = d3
    u2 = q(up(d3, P["u2.W"], P["u2.b"]))
    d2 = cr("d2b", cr("d2a", np.concatenate([u2, e2], axis=3)))
    c["u1.in"] = d2
    u1 = q(up(d2, P["u1.W"], P["u1.b"]))
    d1 = cr("d1b", cr("d1a", np.concatenate([u1, e1], axis=3)))
    c["head.in"] = d1
    y = (d1 @ P["head.W"])[..., 0] + P["head.b"][0]
    return y, c


def backward(P, c, gy, q=None):
    """Gradients of sum(gy * forward(P, x)[0]) for every parameter.

    q (default: identity), as in forward, is applied to the 3^3 convolution
    weights and to every stored activation gradient (the head's and each
    layer's input gradient, and the skip + pooled gradient sums)."""
    q = q or _ident
    G = {}
    d1 = c["head.in"]
    G["head.W"] = np.einsum("zyxi,zyx->i", d1, gy)[:, None]
    G["head.b"] = np.array([gy.sum()])
    g = q(gy[..., None] * P["head.W"][:, 0])

    def crb(name, g_out):
        gz = g_out * (c[name + ".z"] > 0)
        gx, G[name + ".W"], G[name + ".b"] = conv3_backward(c[name + ".in"], q(P[name + ".W"]), gz)
        return q(gx)

    g = crb("d1a", crb("d1b", g))
    c1 = P["u1.W"].shape[2]
    g_u1, g_e1_skip = g[..., :c1], g[..., c1:]
    g_d2, G["u1.W"], G["u1.b"] = up_backward(c["u1.in"], P["u1.W"], g_u1)
    g = crb("d2a", crb("d2b", q(g_d2)))
    c2 = P["u2.W"].shape[2]
    g_u2, g_e2_skip = g[..., :c2], g[..., c2:]
    g_d3, G["u2.W"], G["u2.b"] = up_backward(c["u2.in"], P["u2.W"], g_u2)
    g = crb("d3a", crb("d3b", q(g_d3)))
    c3 = P["u3.W"].shape[2]
    g_u3, g_e3_skip = g[..., :c3], g[..., c3:]
    g_bn, G["u3.W"], G["u3.b"] = up_backward(c["u3.in"], P["u3.W"], g_u3)
    g = crb("bna", crb("bnb", q(g_bn)))
    g = q(pool_backward(c["p3.in"], g) + g_e3_skip)
    g = crb("e3a", crb("e3b", g))
    g = q(pool_backward(c["p2.in"], g) + g_e2_skip)
    g = crb("e2a", crb("e2b", g))
    g = q(pool_backward(c["p1.in"], g) + g_e1_skip)
    crb("e1a", crb("e1b", g))
    return G


def mse(y, t, mask=None):
    """(loss, d loss / d y) for the weighted mean sum m (y - t)^2 / max(sum m, 1)
    (m = mask, 1 if None; a 0/1 mask gives the mean over the masked points)."""
    m = np.ones_like(y) if mask is None else mask.astype(np.float64)
    n = max(m.sum(), 1.0)
    r = y - t
    return float((m * r * r).sum() / n), 2.0 * m * r / n


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
