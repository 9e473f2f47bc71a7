"""GPU network kernels against the FP64 network oracle (oracle/conv.py), and
the warm start's gain over the tanh start.

Tolerances: the GPU multiplies bfloat16 weights by FP32 activations with FP32
accumulation; the oracle uses the same bfloat16-rounded weights in FP64, so
the remaining difference is FP32 rounding (<= 1e-5 of the output scale for
the forward pass, <= 1e-4 for gradients summed over a batch of images)."""
import numpy as np
import pytest

from oracle import conv as C
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1906_11027_amd import sc_lbm as B  # noqa: E402
from paper_1906_11027_amd import warmstart as WS  # noqa: E402


def _dev(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _bf16(w):
    bits = WS._bf16_round(w)
    return bits, (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _stream():
    return torch.cuda.current_stream().cuda_stream


# (5, 7) and (1, 3): images narrower than a 16 x 16 tile plus its halo, whose
# halo coordinates wrap more than one period
SHAPES = [(20, 37), (5, 7), (1, 3)]


@pytest.mark.parametrize("h,w", SHAPES)
@pytest.mark.parametrize("cin,cout", [(5, 32), (32, 32), (32, 1)])
def test_conv_forward(cin, cout, h, w):
    rng = np.random.default_rng(cin + cout)
    bsz = 3
    x = rng.normal(size=(bsz, cin, h, w))
    wt = rng.normal(scale=0.2, size=(cout, cin, 3, 3)).astype(np.float32)
    bias = rng.normal(size=cout).astype(np.float32)
    bits, wq = _bf16(wt)
    xd, out = _dev(x), torch.empty((bsz, cout, h, w), dtype=torch.float32, device="cuda")
    wd = torch.tensor(bits.view(np.int16), device="cuda")
    bd = _dev(bias)
    assert B.lib().sc_nn_conv3x3_fwd(xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), out.data_ptr(), bsz, cin, cout,
                                     h, w, _stream()) == 0
    ref = C.conv_fwd(x.astype(np.float32).astype(np.float64), wq, bias.astype(np.float64))
    err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref))
    say("conv fwd %d->%d %dx%d err %.2e" % (cin, cout, h, w, err))
    assert err < 1e-5


@pytest.mark.parametrize("h,w", [(19, 34), (5, 7), (1, 3)])
@pytest.mark.parametrize("cin,cout", [(5, 32), (32, 32), (32, 1)])
def test_conv_backward(cin, cout, h, w):
    rng = np.random.default_rng(7 + cin + cout)
    bsz = 3
    x = rng.normal(size=(bsz, cin, h, w)).astype(np.float32)
    g = rng.normal(size=(bsz, cout, h, w)).astype(np.float32)
    wt = rng.normal(scale=0.2, size=(cout, cin, 3, 3)).astype(np.float32)
    bits, wq = _bf16(wt)
    gin_ref, gw_ref, gb_ref = C.conv_bwd(x.astype(np.float64), wq, g.astype(np.float64))
    xd, gd = _dev(x), _dev(g)
    wd = torch.tensor(bits.view(np.int16), device="cuda")
    nblk = 37
    scratch = torch.empty(B.lib().sc_nn_bwd_weight_scratch_floats(cin, cout, nblk), device="cuda")
    gw = torch.empty((cout, cin, 3, 3), device="cuda")
    gb = torch.empty(cout, device="cuda")
    assert B.lib().sc_nn_conv3x3_bwd_weight(xd.data_ptr(), gd.data_ptr(), scratch.data_ptr(), nblk, gw.data_ptr(),
                                            gb.data_ptr(), bsz, cin, cout, h, w, _stream()) == 0
    ew = np.max(np.abs(gw.cpu().numpy() - gw_ref)) / np.max(np.abs(gw_ref))
    eb = np.max(np.abs(gb.cpu().numpy() - gb_ref)) / np.max(np.abs(gb_ref))
    say("conv bwd w %d->%d %dx%d err %.2e bias %.2e" % (cin, cout, h, w, ew, eb))
    assert ew < 1e-4 and eb < 1e-4
    if cin == 32:
        gin = torch.empty((bsz, cin, h, w), device="cuda")
        wts = torch.empty(cin * cout * 9, dtype=torch.int16, device="cuda")
        assert B.lib().sc_nn_conv3x3_bwd_data(gd.data_ptr(), wd.data_ptr(), wts.data_ptr(), gin.data_ptr(), bsz, cin,
                                              cout, h, w, _stream()) == 0
        ei = np.max(np.abs(gin.cpu().numpy() - gin_ref)) / np.max(np.abs(gin_ref))
        say("conv bwd data %d->%d err %.2e" % (cin, cout, ei))
        assert ei < 1e-5


def test_conv_items_beyond_one_per_block():
    """The MFMA kernels are persistent: 512 blocks take (image, 16 x 16 tile)
    items in turn.  9 images of 128 x 128 (576 items) make some blocks take
    a second item through the same LDS; forward, weight gradient and
    backward-data against the oracle."""
    rng = np.random.default_rng(11)
    bsz, cin, cout, h, w = 9, 32, 32, 128, 128
    x = rng.normal(size=(bsz, cin, h, w)).astype(np.float32)
    g = rng.normal(size=(bsz, cout, h, w)).astype(np.float32)
    wt = rng.normal(scale=0.2, size=(cout, cin, 3, 3)).astype(np.float32)
    bias = rng.normal(size=cout).astype(np.float32)
    bits, wq = _bf16(wt)
    xd, gd, bd = _dev(x), _dev(g), _dev(bias)
    wd = torch.tensor(bits.view(np.int16), device="cuda")
    out = torch.empty((bsz, cout, h, w), device="cuda")
    assert B.lib().sc_nn_conv3x3_fwd(xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), out.data_ptr(), bsz, cin, cout, h,
                                     w, _stream()) == 0
    ref = C.conv_fwd(x.astype(np.float64), wq, bias.astype(np.float64))
    err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref))
    gin_ref, gw_ref, gb_ref = C.conv_bwd(x.astype(np.float64), wq, g.astype(np.float64))
    nblk = 512
    scratch = torch.empty(B.lib().sc_nn_bwd_weight_scratch_floats(cin, cout, nblk), device="cuda")
    gw = torch.empty((cout, cin, 3, 3), device="cuda")
    gb = torch.empty(cout, device="cuda")
    assert B.lib().sc_nn_conv3x3_bwd_weight(xd.data_ptr(), gd.data_ptr(), scratch.data_ptr(), nblk, gw.data_ptr(),
                                            gb.data_ptr(), bsz, cin, cout, h, w, _stream()) == 0
    ew = np.max(np.abs(gw.cpu().numpy() - gw_ref)) / np.max(np.abs(gw_ref))
    eb = np.max(np.abs(gb.cpu().numpy() - gb_ref)) / np.max(np.abs(gb_ref))
    gin = torch.empty((bsz, cin, h, w), device="cuda")
    wts = torch.empty(cin * cout * 9, dtype=torch.int16, device="cuda")
    assert B.lib().sc_nn_conv3x3_bwd_data(gd.data_ptr(), wd.data_ptr(), wts.data_ptr(), gin.data_ptr(), bsz, cin,
                                          cout, h, w, _stream()) == 0
    ei = np.max(np.abs(gin.cpu().numpy() - gin_ref)) / np.max(np.abs(gin_ref))
    say("conv 576 items: fwd %.2e, weight grad %.2e, bias grad %.2e, data grad %.2e" % (err, ew, eb, ei))
    assert err < 1e-5 and ei < 1e-5
    assert ew < 1e-4 and eb < 1e-4


@pytest.mark.parametrize("h,w,bsz", [(20, 37, 3), (5, 7, 2), (128, 128, 9)])
def test_fused_tanh_passes(h, w, bsz):
    """The convolutions with the tanh fused into their store give what the
    separate passes give: forward then tanh, backward-data then the tanh
    derivative of the layer's input (same operations in the same order)."""
    rng = np.random.default_rng(h + w)
    cin = cout = 32
    x = rng.normal(size=(bsz, cin, h, w)).astype(np.float32)
    y = np.tanh(rng.normal(size=(bsz, cin, h, w))).astype(np.float32)
    g = rng.normal(size=(bsz, cout, h, w)).astype(np.float32)
    bits, _ = _bf16(rng.normal(scale=0.2, size=(cout, cin, 3, 3)).astype(np.float32))
    xd, yd, gd, bd = _dev(x), _dev(y), _dev(g), _dev(rng.normal(size=cout).astype(np.float32))
    wd = torch.tensor(bits.view(np.int16), device="cuda")
    L, st = B.lib(), _stream()
    a, b = torch.empty((bsz, cout, h, w), device="cuda"), torch.empty((bsz, cout, h, w), device="cuda")
    assert L.sc_nn_conv3x3_fwd(xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), a.data_ptr(), bsz, cin, cout, h, w,
                               st) == 0
    assert L.sc_nn_tanh_fwd(a.data_ptr(), a.numel(), st) == 0
    assert L.sc_nn_conv3x3_fwd_tanh(xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), b.data_ptr(), bsz, cin, cout, h, w,
                                    st) == 0
    df = float((a - b).abs().max())
    wts = torch.empty(cin * cout * 9, dtype=torch.int16, device="cuda")
    c, e = torch.empty((bsz, cin, h, w), device="cuda"), torch.empty((bsz, cin, h, w), device="cuda")
    assert L.sc_nn_conv3x3_bwd_data(gd.data_ptr(), wd.data_ptr(), wts.data_ptr(), c.data_ptr(), bsz, cin, cout, h,
                                    w, st) == 0
    assert L.sc_nn_tanh_bwd(yd.data_ptr(), c.data_ptr(), c.numel(), st) == 0
    assert L.sc_nn_conv3x3_bwd_data_tanh(gd.data_ptr(), wd.data_ptr(), wts.data_ptr(), yd.data_ptr(), e.data_ptr(),
                                         bsz, cin, cout, h, w, st) == 0
    db = float((c - e).abs().max())
    say("fused tanh %dx%d: forward max diff %.1e, backward-data max diff %.1e" % (h, w, df, db))
    assert df <= 1e-6 and db <= 1e-6 * float(c.abs().max())
    # one output channel has no fused form (the net's last layer is linear)
    assert L.sc_nn_conv3x3_fwd_tanh(xd.data_ptr(), wd.data_ptr(), bd.data_ptr(), b.data_ptr(), bsz, cin, 1, h, w,
                                    st) == B.SC_E_INVAL


def test_pointwise_kernels():
    rng = np.random.default_rng(3)
    n = 5000
    x = rng.normal(size=n).astype(np.float32)
    xd = _dev(x)
    assert B.lib().sc_nn_tanh_fwd(xd.data_ptr(), n, _stream()) == 0
    y = xd.cpu().numpy()
    assert np.max(np.abs(y - np.tanh(x.astype(np.float64)))) < 2e-7
    g = rng.normal(size=n).astype(np.float32)
    gd = _dev(g)
    assert B.lib().sc_nn_tanh_bwd(xd.data_ptr(), gd.data_ptr(), n, _stream()) == 0
    assert np.allclose(gd.cpu().numpy(), g * (1 - y.astype(np.float64) ** 2), rtol=1e-6, atol=1e-7)
    t = rng.normal(size=n).astype(np.float32)
    part = torch.empty(16, dtype=torch.float64, device="cuda")
    grad = torch.empty(n, device="cuda")
    xd2, td = _dev(x), _dev(t)   # referenced until the kernel has run
    assert B.lib().sc_nn_mse(xd2.data_ptr(), td.data_ptr(), grad.data_ptr(), part.data_ptr(), 16, n,
                             _stream()) == 0
    loss, gref = C.mse(x.astype(np.float64), t.astype(np.float64))
    assert abs(part.cpu().numpy().sum() / n - loss) < 1e-6 * loss
    assert np.allclose(grad.cpu().numpy(), gref, rtol=1e-5, atol=1e-9)
    # Adam, two steps, against the textbook update
    p0 = rng.normal(size=n).astype(np.float32)
    pd, md, vd = _dev(p0), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    bits = torch.empty(n, dtype=torch.int16, device="cuda")
    p, m, v = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t_ in (1, 2):
        gg = rng.normal(size=n).astype(np.float32)
        ggd = _dev(gg)
        assert B.lib().sc_nn_adam(pd.data_ptr(), ggd.data_ptr(), md.data_ptr(), vd.data_ptr(), bits.data_ptr(),
                                  n, 1e-2, 0.9, 0.999, 1e-8, t_, _stream()) == 0
        m = 0.9 * m + 0.1 * gg
        v = 0.999 * v + 0.001 * gg.astype(np.float64) ** 2
        p = p - 1e-2 * (m / (1 - 0.9 ** t_)) / (np.sqrt(v / (1 - 0.999 ** t_)) + 1e-8)
    assert np.max(np.abs(pd.cpu().numpy() - p)) < 1e-5
    assert np.array_equal(bits.cpu().numpy().view(np.uint16), WS._bf16_round(pd.cpu().numpy()))


def test_features():
    prm = np.array([[0.3, -0.2, 0.5, 1.0], [0.1, 0.0, -1.0, -1.0]], dtype=np.float32)
    h, w = 13, 10
    out = torch.empty((2, 5, h, w), device="cuda")
    prmd = _dev(prm)
    assert B.lib().sc_nn_features(prmd.data_ptr(), out.data_ptr(), 2, h, w, 10.0, _stream()) == 0
    o = out.cpu().numpy()
    ref = C.features(prm.astype(np.float64), h, w, 10.0)
    assert np.max(np.abs(o[:, 0] - ref[:, 0])) < 1e-6
    for c in range(4):
        assert np.all(o[:, c + 1] == prm[:, c][:, None, None])


@pytest.mark.parametrize("n", [20, 21])
def test_start_field(n):
    """sc_nn_start_field against the oracle's definition: the average of
    the eight square symmetries of base + resid / scale, clamped, shifted to
    the target mass (FP64 sums on both sides; resid is float32)."""
    rng = np.random.default_rng(n)
    bsz = 3
    resid = rng.normal(scale=3.0, size=(bsz, n, n)).astype(np.float32)
    base = rng.uniform(0.1, 2.0, size=(bsz, n, n))
    mass = base.reshape(bsz, -1).sum(axis=1) + rng.normal(size=bsz)
    out = torch.empty((bsz, n, n), dtype=torch.float64, device="cuda")
    # the inputs stay referenced until the kernel has run: a temporary freed
    # after data_ptr() could be handed to the next allocation on the stream
    rd, bd, md = _dev(resid), _dev(base, torch.float64), _dev(mass, torch.float64)
    rc = B.lib().sc_nn_start_field(rd.data_ptr(), bd.data_ptr(), md.data_ptr(), out.data_ptr(), bsz, n, n, 0.1,
                                   0.05, 2.5, _stream())
    assert rc == 0
    got = out.cpu().numpy()
    for b in range(bsz):
        ref = C.start_field(resid[b].astype(np.float64), base[b], mass[b], 10.0, 0.05, 2.5)
        err = np.max(np.abs(got[b] - ref))
        say("start field n=%d item %d: max err %.2e" % (n, b, err))
        assert err < 1e-7
        assert abs(got[b].sum() - mass[b]) < 1e-10 * abs(mass[b])
    assert B.lib().sc_nn_start_field(rd.data_ptr(), bd.data_ptr(), md.data_ptr(), out.data_ptr(), bsz, n, n + 1,
                                     0.1, 0.05, 2.5, _stream()) == B.SC_E_INVAL


def test_network_gradients_against_oracle():
    h, w, bsz = 20, 18, 2
    net = WS.WarmStartNet(h, w, bsz, seed=4)
    rng = np.random.default_rng(5)
    prm = rng.normal(scale=0.5, size=(bsz, 4))
    net.set_params(prm)
    out = net.forward().cpu().numpy().astype(np.float64)
    x = net.acts[0].cpu().numpy().astype(np.float64)
    tgt = rng.normal(size=(bsz, 1, h, w)).astype(np.float32)
    params = net.weights_numpy()
    acts = C.net_forward(params, x)
    assert np.max(np.abs(out - acts[-1])) < 1e-4 * np.max(np.abs(acts[-1]))
    net.loss_and_grad(_dev(tgt))
    net.backward()
    _, g = C.mse(acts[-1], tgt.astype(np.float64))
    grads = C.net_backward(params, acts, g)
    for li in range(5):
        gw = net.gW[li].cpu().numpy()
        gb = net.gb[li].cpu().numpy()
        ew = np.linalg.norm(gw - grads[li][0]) / np.linalg.norm(grads[li][0])
        eb = np.linalg.norm(gb - grads[li][1]) / np.linalg.norm(grads[li][1])
        say("layer %d grad err w %.2e b %.2e" % (li, ew, eb))
        assert ew < 1e-3 and eb < 1e-3


def test_training_reduces_loss():
    """Fit the net to tanh droplet profiles of the radius encoded in channel 1."""
    h = w = 32
    net = WS.WarmStartNet(h, w, 8, seed=1)
    rng = np.random.default_rng(2)
    inputs, targets = [], []
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    r = np.sqrt((xx - w // 2) ** 2 + (yy - h // 2) ** 2)
    for _ in range(64):
        R = rng.uniform(5, 12)
        inputs.append(WS.normalise(R, -5.0, 1.0, 4))
        targets.append(1.075 - 0.925 * np.tanh(2 * (r - R) / 2.5))
    hist = WS.train(net, inputs, targets, epochs=30, lr=3e-3)
    say("training loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.1 * hist[0]


def test_warm_start_gain_small():
    """Scaled-down warm-start experiment on 64^2 droplets.  What the trained
    net gains over the tanh start: an initial density field several times
    closer to the steady state and, started at rest in the forced sense,
    fewer steps to the steady-state rule (max|u| change < 1e-10, batched FP64
    runs); both starts reach the same steady field."""
    res = WS.run_experiment(n_train=128, n_test=12, side=64, tol=1e-8, epochs=400, batch=16, lr=1e-3,
                            max_steps=80000, obs_every=100, chunk=64, fp64_baseline=2, seed=77, tols=(1e-10,),
                            log=lambda m: None)
    runs = res.pop("runs")["1e-10"]
    say("warm start:", res)
    for name, r in runs.items():
        say("  ", name, r)
    assert res["n_test"] >= 8
    assert runs["learned"]["converged"] >= res["n_test"] - 1
    assert res["loss_last"] < 0.05 * res["loss_first"]
    assert res["err_rms_median"]["learned"] < 0.5 * res["err_rms_median"]["tanh"]
    assert runs["learned"]["steps_mean"] < 0.9 * runs["tanh"]["steps_mean"]
    # both starts are symmetric, so they settle on the same droplet (no
    # translation to align): the FP64 steady fields agree to 1e-5 of rho
    assert runs["steady_fields_max_abs_diff_median"] < 1e-5 * 2.0
