"""Pins for the FP64 network oracle (oracle/conv.py): the convolution against
a nested-loop evaluation of its defining sum, and every gradient against
central finite differences of the loss."""
import numpy as np

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


def test_square_images_brute_force():
    """Each image against an explicit coordinate map (odd and even sides)."""
    for n in (5, 6):
        c = n // 2
        a = np.arange(n * n, dtype=float).reshape(n, n) ** 1.5
        ims = C.square_images(a)
        assert len(ims) == 8
        maps = []
        for tr in (False, True):
            for fi in (False, True):
                for fj in (False, True):
                    def m(i, j, tr=tr, fi=fi, fj=fj):
                        if fi:
                            i = (2 * c - i) % n
                        if fj:
                            j = (2 * c - j) % n
                        return (j, i) if tr else (i, j)
                    maps.append(m)
        for im, m in zip(ims, maps):
            for i in range(n):
                for j in range(n):
                    assert im[i, j] == a[m(i, j)]
        # the images form a group: every one is distinct for a generic field
        assert len({im.tobytes() for im in ims}) == 8


def test_start_field_keeps_a_symmetric_field_and_mass():
    from workload import droplet_rho
    base = droplet_rho((32, 32), 9)
    out = C.start_field(np.zeros((32, 32)), base, base.sum(), 10.0, 0.05, 2.5)
    assert np.max(np.abs(out - base)) < 1e-14
    # a perturbation odd about the centre node on the periodic grid averages
    # away; the mass is met
    x = np.sin(2 * np.pi * (np.arange(32) - 16.0) / 32)[:, None] * np.ones(32)[None]
    out = C.start_field(10.0 * 0.01 * x, base, base.sum() + 3.0, 10.0, 0.05, 2.5)
    assert np.max(np.abs(out - (base + 3.0 / 1024))) < 1e-14
    # clamping happens before the mass shift
    out = C.start_field(np.full((32, 32), -40.0), base, base.sum(), 10.0, 0.05, 2.5)
    assert abs(out.sum() - base.sum()) < 1e-10 and np.ptp(out) < 1e-12


def test_features_definition():
    prm = np.array([[0.7, 0.1, -0.2, 0.3]])
    f = C.features(prm, 9, 12, 10.0)
    assert f.shape == (1, 5, 9, 12)
    # node (y, x) = (4, 6) is the centre; (0, 0) is sqrt(4^2 + 6^2) away
    assert abs(f[0, 0, 4, 6] + 0.7) < 1e-15
    assert abs(f[0, 0, 0, 0] - (np.sqrt(52.0) / 10.0 - 0.7)) < 1e-15
    assert np.all(f[0, 3] == -0.2)
