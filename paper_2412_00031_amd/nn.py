"""Python binding of the warm-start network ABI (include/nn.h): argument
marshalling over torch device tensors.  Activations are torch.bfloat16 tensors
(used as storage only), parameters and gradients float32; every computation
runs in libtt's kernels.
"""
import ctypes

import torch

from . import _lib
from .api import _dev, _grid, _stream

_BF = torch.bfloat16
_F32 = torch.float32


def _p(t, name, dtype):
    return _dev(t, name, dtype)


def _ptr_or_null(t, name, dtype):
    return _p(t, name, dtype) if t is not None else ctypes.c_void_p(0)


def _st(t):
    return _stream(t.device)


def _call(fn, *args):
    _lib.check(fn(*args))


def cfg(ch=(16, 32, 32, 64), in_ch=4):
    c = _lib.NNUnetCfg()
    for i in range(4):
        c.ch[i] = int(ch[i])
    c.in_ch = int(in_ch)
    return c


def to_bf16(x, out=None):
    lib = _lib.load()
    out = torch.empty(x.shape, dtype=_BF, device=x.device) if out is None else out
    _call(lib.nn_to_bf16, _p(x, "x", _F32), x.numel(), _p(out, "out", _BF), _st(x))
    return out


def from_bf16(x, out=None):
    lib = _lib.load()
    out = torch.empty(x.shape, dtype=_F32, device=x.device) if out is None else out
    _call(lib.nn_from_bf16, _p(x, "x", _BF), x.numel(), _p(out, "out", _F32), _st(x))
    return out


def conv3_pack(W, flip=False):
    """W [27, cin, cout] float32 -> bf16 fragments (flip: data-gradient set)."""
    lib = _lib.load()
    _, cin, cout = W.shape
    kb = cout // 16 if flip else (cin + 15) // 16
    nb = cin // 16 if flip else cout // 16
    frag = torch.empty(27 * kb * nb * 256, dtype=_BF, device=W.device)
    _call(lib.nn_conv3_pack, _p(W, "W", _F32), int(cin), int(cout), int(bool(flip)), _p(frag, "frag", _BF), _st(W))
    return frag


def conv3_fwd(x, cin, frag, bias, cout, relu, y, cx_off=0, cy_off=0):
    """x [nb, D, H, W, cx_total], y [nb, D, H, W, cy_total] (bf16)."""
    lib = _lib.load()
    nb, D, H, W, cxt = x.shape
    _call(lib.nn_conv3_fwd, _p(x, "x", _BF), nb, D, H, W, cxt, int(cx_off), int(cin), _p(frag, "frag", _BF),
          _ptr_or_null(bias, "bias", _F32), int(cout), int(bool(relu)), _p(y, "y", _BF), y.shape[-1], int(cy_off),
          _st(x))
    return y


def conv3_wgrad(x, cin, gz, cout, cx_off=0, cg_off=0, with_bias=True):
    lib = _lib.load()
    nb, D, H, W, cxt = x.shape
    gW = torch.empty((27, cin, cout), dtype=_F32, device=x.device)
    gb = torch.empty(cout, dtype=_F32, device=x.device) if with_bias else None
    nwork = lib.nn_conv3_wgrad_work(nb, D, H, W, int(cin), int(cout))
    work = torch.empty(max(nwork // 4, 1), dtype=_F32, device=x.device)
    _call(lib.nn_conv3_wgrad, _p(x, "x", _BF), nb, D, H, W, cxt, int(cx_off), int(cin), _p(gz, "gz", _BF),
          gz.shape[-1], int(cg_off), int(cout), _p(gW, "gW", _F32), _ptr_or_null(gb, "gb", _F32),
          _p(work, "work", _F32), work.numel() * 4, _st(x))
    return gW, gb


def relu_mask(g, y, c, g_out, c_off=0, co_off=0):
    lib = _lib.load()
    npos = g.numel() // g.shape[-1]
    _call(lib.nn_relu_mask, _p(g, "g", _BF), _p(y, "y", _BF), npos, g.shape[-1], int(c_off), int(c),
          _p(g_out, "g_out", _BF), g_out.shape[-1], int(co_off), _st(g))
    return g_out


def pool_fwd(x, c, c_off=0):
    lib = _lib.load()
    nb, D, H, W, ct = x.shape
    y = torch.empty((nb, D // 2, H // 2, W // 2, c), dtype=_BF, device=x.device)
    _call(lib.nn_pool_fwd, _p(x, "x", _BF), nb, D, H, W, ct, int(c_off), int(c), _p(y, "y", _BF), _st(x))
    return y


def pool_bwd(x, gy, c, gx, c_off=0, accumulate=False):
    lib = _lib.load()
    nb, D, H, W, ct = x.shape
    _call(lib.nn_pool_bwd, _p(x, "x", _BF), _p(gy, "gy", _BF), nb, D, H, W, ct, int(c_off), int(c), _p(gx, "gx", _BF),
          int(bool(accumulate)), _st(x))
    return gx


def up_fwd(x, Wu, b, y, cy_off=0):
    lib = _lib.load()
    nb, D, H, W, cin = x.shape
    cout = Wu.shape[2]
    _call(lib.nn_up_fwd, _p(x, "x", _BF), nb, D, H, W, cin, _p(Wu, "Wu", _F32), _p(b, "b", _F32), cout,
          _p(y, "y", _BF), y.shape[-1], int(cy_off), _st(x))
    return y


def up_bwd(x, gy, Wu, cg_off=0, with_gx=True):
    lib = _lib.load()
    nb, D, H, W, cin = x.shape
    cout = Wu.shape[2]
    gx = torch.empty_like(x) if with_gx else None
    gW = torch.empty_like(Wu)
    gb = torch.empty(cout, dtype=_F32, device=x.device)
    nwork = lib.nn_up_wgrad_work(nb, D, H, W, cin, cout)
    work = torch.empty(max(nwork // 4, 1), dtype=_F32, device=x.device)
    _call(lib.nn_up_bwd, _p(x, "x", _BF), _p(gy, "gy", _BF), nb, D, H, W, cin, cout, gy.shape[-1], int(cg_off),
          _p(Wu, "Wu", _F32), _ptr_or_null(gx, "gx", _BF), _p(gW, "gW", _F32), _p(gb, "gb", _F32),
          _p(work, "work", _F32), work.numel() * 4, _st(x))
    return gx, gW, gb


def head_fwd(x, w, b):
    lib = _lib.load()
    cin = x.shape[-1]
    npos = x.numel() // cin
    y = torch.empty(x.shape[:-1], dtype=_F32, device=x.device)
    _call(lib.nn_head_fwd, _p(x, "x", _BF), npos, cin, _p(w, "w", _F32), _p(b, "b", _F32), _p(y, "y", _F32), _st(x))
    return y


def head_bwd(x, gy, w):
    lib = _lib.load()
    cin = x.shape[-1]
    npos = x.numel() // cin
    gx = torch.empty_like(x)
    gw = torch.empty(cin, dtype=_F32, device=x.device)
    gb = torch.empty(1, dtype=_F32, device=x.device)
    nwork = lib.nn_head_work(npos, cin)
    work = torch.empty(max(nwork // 4, 1), dtype=_F32, device=x.device)
    _call(lib.nn_head_bwd, _p(x, "x", _BF), _p(gy, "gy", _F32), npos, cin, _p(w, "w", _F32), _p(gx, "gx", _BF),
          _p(gw, "gw", _F32), _p(gb, "gb", _F32), _p(work, "work", _F32), work.numel() * 4, _st(x))
    return gx, gw, gb


def mse(y, t, mask=None, loss=None, gy=None):
    """Returns (loss buffer: [0] mean, [1] count, rest scratch; gy)."""
    lib = _lib.load()
    loss = torch.empty(_lib.NN_MSE_LOSS_FLOATS, dtype=_F32, device=y.device) if loss is None else loss
    gy = torch.empty_like(y) if gy is None else gy
    _call(lib.nn_mse, _p(y, "y", _F32), _p(t, "t", _F32), _ptr_or_null(mask, "mask", _F32), y.numel(),
          _p(loss, "loss", _F32), _p(gy, "gy", _F32), _st(y))
    return loss, gy


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    lib = _lib.load()
    _call(lib.nn_adam, _p(p, "p", _F32), _p(g, "g", _F32), _p(m, "m", _F32), _p(v, "v", _F32), p.numel(), int(step),
          float(lr), float(beta1), float(beta2), float(eps), _st(p))


# ----------------------------------------------------------------- U-Net
def unet_sizes(c):
    lib = _lib.load()
    return lib.nn_unet_nparams(ctypes.byref(c)), lib.nn_unet_nfrag(ctypes.byref(c))


def unet_workspace(c, nbatch, D, H, W, train, device):
    lib = _lib.load()
    n = lib.nn_unet_workspace(ctypes.byref(c), nbatch, D, H, W, int(bool(train)))
    if n == 0:
        raise ValueError("invalid U-Net configuration or sizes")
    return torch.empty(n, dtype=torch.uint8, device=device)


def unet_pack(c, params, frag):
    lib = _lib.load()
    _call(lib.nn_unet_pack, ctypes.byref(c), _p(params, "params", _F32), _p(frag, "frag", _BF), _st(params))


def unet_forward(c, params, frag, x, y, ws, train):
    lib = _lib.load()
    nb, D, H, W, _ = x.shape
    _call(lib.nn_unet_forward, ctypes.byref(c), _p(params, "params", _F32), _p(frag, "frag", _BF), _p(x, "x", _BF),
          nb, D, H, W, _p(y, "y", _F32), _dev(ws, "ws", torch.uint8), ws.numel(), int(bool(train)), _st(x))
    return y


def unet_backward(c, params, frag, x, gy, grad, ws):
    lib = _lib.load()
    nb, D, H, W, _ = x.shape
    _call(lib.nn_unet_backward, ctypes.byref(c), _p(params, "params", _F32), _p(frag, "frag", _BF), _p(x, "x", _BF),
          _p(gy, "gy", _F32), nb, D, H, W, _p(grad, "grad", _F32), _dev(ws, "ws", torch.uint8), ws.numel(), _st(x))
    return grad


# ------------------------------------------------------------ warm start
def warm_features(grid, s, xi, eta, src, par, stride, dims, out=None):
    lib = _lib.load()
    nsrc = int(src.shape[0])
    D, H, W = dims
    out = torch.empty((nsrc, D, H, W, 16), dtype=_BF, device=s.device) if out is None else out
    g = _grid(grid)
    f64 = torch.float64
    _call(lib.nn_warm_features, ctypes.byref(g), _p(s, "s", f64), _p(xi, "xi", f64), _p(eta, "eta", f64), nsrc,
          _p(src, "src", f64), _p(par, "par", f64), int(stride), D, H, W, _p(out, "feat", _BF), _st(s))
    return out


def warm_target(grid, tau, stride, dims, target=None, mask=None, with_mask=True):
    lib = _lib.load()
    nsrc = int(tau.shape[0])
    D, H, W = dims
    target = torch.empty((nsrc, D, H, W), dtype=_F32, device=tau.device) if target is None else target
    if with_mask and mask is None:
        mask = torch.empty_like(target)
    g = _grid(grid)
    _call(lib.nn_warm_target, ctypes.byref(g), nsrc, _p(tau, "tau", torch.float64), int(stride), D, H, W,
          _p(target, "target", _F32), _ptr_or_null(mask, "mask", _F32), _st(tau))
    return target, mask


def warm_init(grid, pred, stride, out=None):
    lib = _lib.load()
    nsrc, D, H, W = pred.shape
    n = grid["n"]
    N = int(n[0]) * int(n[1]) * int(n[2])
    out = torch.empty((nsrc, N), dtype=torch.float64, device=pred.device) if out is None else out
    g = _grid(grid)
    _call(lib.nn_warm_init, ctypes.byref(g), nsrc, _p(pred, "pred", _F32), int(stride), D, H, W,
          _p(out, "tau_init", torch.float64), _st(pred))
    return out
