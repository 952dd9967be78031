"""Learned warm start of the factored Eikonal solve.

A 3-D U-Net maps (s, xi, eta, distance to the source), sampled on every
``stride``-th node of the solver grid, to tau - 1 (tau the factor of T = T0 tau,
Sec. 3.1).  Its prediction, interpolated back to the grid, is the initial tau of
the fast sweeping iteration of Eq. (4); the sweeps then run to the same
tolerance as from tau = 1, so the network changes the iteration count, not the
accuracy the solver is held to.  The network is trained on converged fields
that the solver itself produces on random smooth models.

Every computation (features, network layers, loss, optimiser, interpolation,
solves) runs in libtt's kernels; this module allocates buffers and orders calls.
"""
import math
import os
import time

import numpy as np
import torch

from . import api, nn
from . import workloads as W

CH = (16, 32, 32, 64)
IN_CH = 4
_BF = torch.bfloat16
_F32 = torch.float32


def param_layout(ch=CH, in_ch=IN_CH):
    """[(name, shape, offset)] of the flat parameter array (include/nn.h order)."""
    c1, c2, c3, c4 = ch
    convs = [("e1a", in_ch, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2), ("e3a", c2, c3),
             ("e3b", c3, c3), ("bna", c3, c4), ("bnb", c4, c4), ("d3a", 2 * c3, c3), ("d3b", c3, c3),
             ("d2a", 2 * c2, c2), ("d2b", c2, c2), ("d1a", 2 * c1, c1), ("d1b", c1, c1)]
    ups = [("u3", c4, c3), ("u2", c3, c2), ("u1", c2, c1)]
    out, off = [], 0
    for name, ci, co in convs:
        out.append((name + ".W", (27, ci, co), off))
        off += 27 * ci * co
        out.append((name + ".b", (co,), off))
        off += co
    for name, ci, co in ups:
        out.append((name + ".W", (8, ci, co), off))
        off += 8 * ci * co
        out.append((name + ".b", (co,), off))
        off += co
    out.append(("head.W", (c1, 1), off))
    off += c1
    out.append(("head.b", (1,), off))
    off += 1
    return out, off


def init_params(seed, ch=CH, in_ch=IN_CH):
    """He-normal initial weights (zero biases) as a flat float32 numpy array."""
    rng = np.random.default_rng(seed)
    lay, n = param_layout(ch, in_ch)
    flat = np.zeros(n, dtype=np.float32)
    for name, shape, off in lay:
        if name.endswith(".b"):
            continue
        if name == "head.W":
            std = math.sqrt(1.0 / shape[0])
        elif shape[0] == 27:
            std = math.sqrt(2.0 / (27 * shape[1]))
        else:
            std = math.sqrt(2.0 / shape[1])
        flat[off:off + int(np.prod(shape))] = rng.standard_normal(int(np.prod(shape))) * std
    return flat


def coarse_dims(grid, stride):
    """Coarse node counts rounded up to multiples of 8 (the U-Net's pooling depth)."""
    return tuple(int(-(-((int(n) - 1) // stride + 1) // 8) * 8) for n in grid["n"])


class UNet:
    """Parameters, fragments, optimiser state and workspaces of one network."""

    def __init__(self, device, ch=CH, in_ch=IN_CH, seed=0, params=None):
        self.ch, self.in_ch = tuple(int(c) for c in ch), int(in_ch)
        self.cfg = nn.cfg(self.ch, self.in_ch)
        self.nparams, self.nfrag = nn.unet_sizes(self.cfg)
        if self.nparams == 0:
            raise ValueError(f"invalid U-Net channels {ch}")
        self.device = torch.device(device)
        flat = init_params(seed, ch, in_ch) if params is None else np.asarray(params, dtype=np.float32)
        if flat.size != self.nparams:
            raise ValueError(f"parameter count {flat.size} != {self.nparams}")
        self.params = torch.as_tensor(flat, device=self.device).contiguous()
        self.frag = torch.empty(self.nfrag, dtype=_BF, device=self.device)
        self.grad = torch.zeros(self.nparams, dtype=_F32, device=self.device)
        self.m = torch.zeros(self.nparams, dtype=_F32, device=self.device)
        self.v = torch.zeros(self.nparams, dtype=_F32, device=self.device)
        self.step = 0
        self._ws = {}
        self.pack()

    def pack(self):
        nn.unet_pack(self.cfg, self.params, self.frag)

    def workspace(self, nbatch, dims, train):
        key = (nbatch, tuple(dims), bool(train))
        ws = self._ws.get(key)
        if ws is None:
            ws = nn.unet_workspace(self.cfg, nbatch, *dims, train, self.device)
            self._ws[key] = ws
        return ws

    def forward(self, x, train=False, y=None):
        nb, D, H, Wd, _ = x.shape
        y = torch.empty((nb, D, H, Wd), dtype=_F32, device=x.device) if y is None else y
        ws = self.workspace(nb, (D, H, Wd), train)
        nn.unet_forward(self.cfg, self.params, self.frag, x, y, ws, train)
        return y

    def backward(self, x, gy):
        nb, D, H, Wd, _ = x.shape
        ws = self.workspace(nb, (D, H, Wd), True)
        nn.unet_backward(self.cfg, self.params, self.frag, x, gy, self.grad, ws)
        return self.grad

    def adam_step(self, lr):
        self.step += 1
        nn.adam(self.params, self.grad, self.m, self.v, self.step, lr)
        self.pack()

    def state(self):
        return {"params": self.params.cpu().numpy(), "ch": np.asarray(self.ch, dtype=np.int32),
                "in_ch": np.asarray([self.in_ch], dtype=np.int32)}

    def save(self, path, **meta):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        extra = {k: np.asarray(v) for k, v in meta.items()}
        np.savez(path, **self.state(), **extra)

    @classmethod
    def load(cls, path, device):
        with np.load(path) as z:
            return cls(device, ch=tuple(int(c) for c in z["ch"]), in_ch=int(z["in_ch"][0]), params=z["params"])


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_sph101.npz")


class WarmStart:
    """tau_init for a batch of sources from a trained network."""

    def __init__(self, net, grid, stride=2, chunk=32):
        self.net, self.grid, self.stride, self.chunk = net, grid, int(stride), int(chunk)
        self.dims = coarse_dims(grid, self.stride)

    def predict(self, s, xi, eta, src, par, out=None):
        nsrc = int(src.shape[0])
        n = self.grid["n"]
        N = int(n[0]) * int(n[1]) * int(n[2])
        out = torch.empty((nsrc, N), dtype=torch.float64, device=s.device) if out is None else out
        for q0 in range(0, nsrc, self.chunk):
            q1 = min(nsrc, q0 + self.chunk)
            feat = nn.warm_features(self.grid, s, xi, eta, src[q0:q1], par[q0:q1], self.stride, self.dims)
            pred = self.net.forward(feat)
            nn.warm_init(self.grid, pred, self.stride, out=out[q0:q1])
        return out


# ------------------------------------------------------------ training data
def training_model(grid, seed):
    """One random smooth model of the kind the solver meets: slowness
    s_bg(depth) (1 + a g_s) with a Gaussian random field g_s of random
    correlation length (8-20 km) and amplitude (5-12 %), azimuthal xi, eta of
    amplitude 0.02-0.05, and sources at uneven depths."""
    rng = np.random.default_rng(seed)
    d = W.depth_of(grid)
    s_bg = (1.0 / (6.0 + 0.02 * d))[:, None, None]
    sp = W.grid_spacing_km(grid)
    corr = rng.uniform(8.0, 20.0)
    amp = rng.uniform(0.05, 0.12)
    aa = rng.uniform(0.02, 0.05)
    gs = W.gaussian_random_field(grid["n"], sp, corr, rng)
    gx = W.gaussian_random_field(grid["n"], sp, corr, rng)
    ge = W.gaussian_random_field(grid["n"], sp, corr, rng)
    return np.ascontiguousarray(s_bg * (1.0 + amp * gs)), aa * gx, aa * ge, rng


def build_training_set(grid, nmodels, nsrc_per_model, seed, kappa=1.05, tol=1e-6, stride=2, device="cuda",
                       log=print):
    """Features and targets on the coarse nodes for nmodels x nsrc_per_model
    solver fields, stored in a fixed shuffled order (so that consecutive blocks
    mix models)."""
    dims = coarse_dims(grid, stride)
    ns = nmodels * nsrc_per_model
    feats = torch.empty((ns,) + dims + (16,), dtype=_BF, device=device)
    targ = torch.empty((ns,) + dims, dtype=_F32, device=device)
    mask = None
    slot = np.random.default_rng(seed + 1).permutation(ns)
    iters = []
    t0 = time.time()
    for mi in range(nmodels):
        s, xi, eta, rng = training_model(grid, seed + 1000 * (mi + 1))
        src = W.random_sources(grid, nsrc_per_model, (2.0, 95.0), rng)
        dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
        s_d, xi_d, eta_d, src_d = dev(s), dev(xi), dev(eta), dev(src)
        par = api.source_params(grid, s_d, xi_d, eta_d, src_d)
        tau, st = api.forward(grid, s_d, xi_d, eta_d, src_d, par, tol, 5000, kappa, poll=True)
        f = nn.warm_features(grid, s_d, xi_d, eta_d, src_d, par, stride, dims)
        t, m = nn.warm_target(grid, tau, stride, dims, with_mask=mask is None)
        if mask is None:
            mask = m[0].clone()
        for q in range(nsrc_per_model):
            k = int(slot[mi * nsrc_per_model + q])
            feats[k].copy_(f[q])
            targ[k].copy_(t[q])
        iters.extend(int(v) for v in st.cpu().tolist())
        if log and (mi + 1) % max(1, nmodels // 10) == 0:
            log(f"training set: {mi + 1}/{nmodels} models, {time.time() - t0:.1f} s, "
                f"mean forward iterations {np.mean(np.abs(iters)):.1f}")
    return dict(feats=feats, targ=targ, mask=mask, dims=dims, stride=stride, iters=iters)


def train(net, data, epochs, batch=8, lr=2e-3, lr_min=5e-5, seed=0, log=print, val_frac=0.05):
    """Adam with cosine learning-rate decay on the masked MSE; returns the
    history of (epoch, train loss, validation loss)."""
    feats, targ, mask1 = data["feats"], data["targ"], data["mask"]
    ns = int(feats.shape[0])
    nval = max(batch, int(round(ns * val_frac)) // batch * batch)
    ntr = (ns - nval) // batch * batch
    dims = data["dims"]
    mask = mask1.expand((batch,) + dims).contiguous()
    loss_buf = torch.empty(2 + 2 * 1024, dtype=_F32, device=feats.device)
    gy = torch.empty((batch,) + dims, dtype=_F32, device=feats.device)
    rng = np.random.default_rng(seed)
    nblk = ntr // batch
    total = epochs * nblk
    hist = []
    step = 0
    for ep in range(epochs):
        order = rng.permutation(nblk)
        acc, cnt = 0.0, 0
        for b in order:
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / max(1, total)))
            x = feats[b * batch:(b + 1) * batch]
            t = targ[b * batch:(b + 1) * batch]
            y = net.forward(x, train=True)
            nn.mse(y, t, mask, loss=loss_buf, gy=gy)
            net.backward(x, gy)
            net.adam_step(lr_t)
            step += 1
            if cnt < 16 or step % 8 == 0:
                acc += float(loss_buf[0])
                cnt += 1
        vl = evaluate(net, data, ntr, ns, batch, mask, loss_buf, gy)
        hist.append((ep, acc / max(cnt, 1), vl))
        if log:
            log(f"epoch {ep + 1}/{epochs}: train mse {acc / max(cnt, 1):.5f}  validation mse {vl:.5f}")
    return hist


def evaluate(net, data, lo, hi, batch, mask, loss_buf, gy):
    feats, targ = data["feats"], data["targ"]
    tot, n = 0.0, 0
    for b0 in range(lo, hi - batch + 1, batch):
        y = net.forward(feats[b0:b0 + batch])
        nn.mse(y, targ[b0:b0 + batch], mask, loss=loss_buf, gy=gy)
        tot += float(loss_buf[0])
        n += 1
    return tot / max(n, 1)
