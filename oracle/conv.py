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
