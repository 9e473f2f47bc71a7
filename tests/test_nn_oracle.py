"""Pins for the FP64 network oracle (oracle/conv.py): the convolution against
a nested-loop evaluation of its defining sum, and every gradient against
central finite differences of the loss."""
import numpy as np
import pytest

from oracle import conv as C


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 5, 4))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    assert np.allclose(C.conv_fwd(x, w, b), C.conv_brute(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv_delta_input_gives_kernel():
    """A unit impulse at (y0, x0) yields out[y0 - dy, x0 - dx] = w[dy+1, dx+1]."""
    x = np.zeros((1, 1, 7, 6))
    x[0, 0, 3, 2] = 1.0
    w = np.arange(9.0).reshape(1, 1, 3, 3) + 1.0
    out = C.conv_fwd(x, w)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            assert out[0, 0, 3 - dy, 2 - dx] == w[0, 0, dy + 1, dx + 1]


def _fd_check(params, x, tgt, eps=1e-6):
    acts = C.net_forward(params, x)
    _, g = C.mse(acts[-1], tgt)
    grads = C.net_backward(params, acts, g)
    rng = np.random.default_rng(1)
    worst = 0.0
    for li, (w, b) in enumerate(params):
        for arr, garr in ((w, grads[li][0]), (b, grads[li][1])):
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + eps
                lp = C.mse(C.net_forward(params, x)[-1], tgt)[0]
                arr[idx] = old - eps
                lm = C.mse(C.net_forward(params, x)[-1], tgt)[0]
                arr[idx] = old
                fd = (lp - lm) / (2 * eps)
                worst = max(worst, abs(fd - garr[idx]) / max(abs(fd), 1e-8))
    return worst


def test_net_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    ch = [5, 4, 4, 4, 4, 1]
    params = [(rng.normal(scale=0.4, size=(ch[i + 1], ch[i], 3, 3)), rng.normal(scale=0.1, size=ch[i + 1]))
              for i in range(5)]
    x = rng.normal(size=(2, 5, 6, 5))
    tgt = rng.normal(size=(2, 1, 6, 5))
    assert _fd_check(params, x, tgt) < 1e-6
