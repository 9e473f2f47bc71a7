"""FP64 CPU oracle for the warm-start network (not part of the paper's method).

TEST INFRASTRUCTURE: imported only by tests/ (gradient checks of the GPU
network kernels) and never by the GPU path.

Definitions (NCHW arrays, circular padding):
    conv:   out[b, o, y, x] = bias[o] + sum_{i, dy, dx} w[o, i, dy+1, dx+1] in[b, i, y+dy, x+dx]
    gradients follow from the chain rule on that sum:
            gin[b, i, q]  = sum_{o, dy, dx} w[o, i, dy+1, dx+1] gout[b, o, q - (dy, dx)]
            gw[o, i, k]   = sum_{b, p} gout[b, o, p] in[b, i, p + d_k]
            gbias[o]      = sum_{b, p} gout[b, o, p]
    net:    five 3x3 convolutions, tanh after the first four.
    loss:   mean squared error.
    input:  channel 0 = |node - (w/2, h/2)| / scale_r - params[0], channels
            1..4 = params broadcast.
    start:  the initial field of a learned start: the average over the eight
            symmetries of the square about node (n/2, n/2) of
            base + resid / scale, clamped, then shifted to a given mass.
"""
import numpy as np

OFFS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]   # k = 3 (dy+1) + (dx+1)


def shifted(x, dy, dx):
    """x[..., y+dy, x+dx] with periodic wrap."""
    return np.roll(np.roll(x, -dy, axis=-2), -dx, axis=-1)


def conv_fwd(x, w, b=None):
    bsz, cin, h, wd = x.shape
    cout = w.shape[0]
    out = np.zeros((bsz, cout, h, wd))
    for k, (dy, dx) in enumerate(OFFS):
        xs = shifted(x, dy, dx)
        out += np.einsum("oi,bihw->bohw", w[:, :, k // 3, k % 3], xs)
    if b is not None:
        out += b[None, :, None, None]
    return out


def conv_bwd(x, w, gout):
    """(gin, gw, gbias) of conv_fwd at input x and weights w."""
    gin = np.zeros_like(x)
    gw = np.zeros_like(w)
    for k, (dy, dx) in enumerate(OFFS):
        gin += shifted(np.einsum("oi,bohw->bihw", w[:, :, k // 3, k % 3], gout), -dy, -dx)
        gw[:, :, k // 3, k % 3] = np.einsum("bohw,bihw->oi", gout, shifted(x, dy, dx))
    gb = gout.sum(axis=(0, 2, 3))
    return gin, gw, gb


def conv_brute(x, w, b):
    """Nested-loop evaluation of the convolution sum (tiny inputs only)."""
    bsz, cin, h, wd = x.shape
    cout = w.shape[0]
    out = np.zeros((bsz, cout, h, wd))
    for n in range(bsz):
        for o in range(cout):
            for y in range(h):
                for xx in range(wd):
                    s = b[o]
                    for i in range(cin):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                s += w[o, i, dy + 1, dx + 1] * x[n, i, (y + dy) % h, (xx + dx) % wd]
                    out[n, o, y, xx] = s
    return out


def net_forward(params, x):
    """params: list of (w, b); returns list of activations [x, a1, ..., a5]."""
    acts = [x]
    for li, (w, b) in enumerate(params):
        z = conv_fwd(acts[-1], w, b)
        acts.append(np.tanh(z) if li < len(params) - 1 else z)
    return acts


def mse(out, tgt):
    return float(np.mean((out - tgt) ** 2)), 2.0 * (out - tgt) / out.size


def net_backward(params, acts, gout):
    """Gradients [(gw, gb)] of every layer given d loss / d output."""
    grads = [None] * len(params)
    g = gout
    for li in range(len(params) - 1, -1, -1):
        w, b = params[li]
        if li < len(params) - 1:
            g = g * (1.0 - acts[li + 1] ** 2)
        gin, gw, gb = conv_bwd(acts[li], w, g)
        grads[li] = (gw, gb)
        g = gin
    return grads


def features(params, h, w, scale_r):
    """params [B][4] -> input [B][5][h][w]."""
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    r = np.sqrt((xx - w // 2) ** 2.0 + (yy - h // 2) ** 2.0) / scale_r
    params = np.asarray(params, dtype=np.float64)
    out = np.empty((len(params), 5, h, w))
    for b, p in enumerate(params):
        out[b, 0] = r - p[0]
        for c in range(4):
            out[b, c + 1] = p[c]
    return out


def square_images(a):
    """The eight images of an n x n field under the symmetries of the square
    about node (c, c), c = n // 2: index i -> 2c - i (mod n) on either axis,
    and the transpose."""
    n = a.shape[0]
    c = n // 2
    m = (2 * c - np.arange(n)) % n
    out = []
    for t in (a, a.T):
        for fi in (False, True):
            for fj in (False, True):
                im = t[m] if fi else t
                out.append(im[:, m] if fj else im)
    return out


def start_field(resid, base, mass, scale, lo, hi):
    """resid, base [n][n]; returns the learned start's initial density."""
    v = base + np.asarray(resid, dtype=np.float64) / scale
    v = np.mean(square_images(v), axis=0)
    v = np.clip(v, lo, hi)
    return v + (mass - v.sum()) / v.size
