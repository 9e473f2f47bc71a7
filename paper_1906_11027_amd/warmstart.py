"""Learned warm start for droplet runs (an addition to the paper's method).

A five-layer 3x3 convolutional net (5 -> 32 -> 32 -> 32 -> 32 -> 1 channels,
tanh between layers, circular padding, bfloat16 weights with FP32
accumulation) maps the droplet parameters (R, G, tau, stencil order,
broadcast as channels) plus the radial coordinate grid (distance to the
centre relative to R) to the steady density field.  It is trained on the
residual between the steady field and the usual tanh start (scaled by
TARGET_SCALE), so an untrained net reproduces the tanh start and training
moves it towards the steady state.

The start handed to the iteration (sc_nn_start_field) is the prediction
averaged over the eight symmetries of the square about the droplet centre
(the steady state of a centred droplet has that symmetry; any asymmetric
error would seed a slowly decaying shape mode), clamped to a physical range
and shifted to the mass of the tanh start (mass is conserved by the step,
so the steady state is fixed by it).  The populations start at rest in the
forced sense (SC_INIT_REST: zero (sum f c + F/2) / rho), so the interface
force of a nearly steady density does not launch a velocity impulse.  The
lattice Boltzmann iteration still runs to its own steady state and alone
decides when it is reached.

Every arithmetic step runs in the library's kernels (sc_nn_* for the net
and the start field, sc_lbm_batch_* for the data); torch only allocates
device memory and provides the stream.  There is no CPU fallback.
"""
import math
import time

import numpy as np

from . import sc_lbm as B

CHANNELS = [5, 32, 32, 32, 32, 1]
# radius and radial coordinate in units of ten nodes (a few interface widths),
# so r - R is of order one across the interface
SCALE_R = 10.0
RHO_CLAMP = (0.05, 2.5)
TARGET_SCALE = 10.0


def normalise(R, G, tau, order):
    """Parameters as the net sees them (roughly unit range near the interface)."""
    return [R / SCALE_R, (G + 5.0) / 0.5, (tau - 1.0) / 0.2, (order - 7.0) / 3.0]


def _bf16_round(a):
    """numpy float32 -> nearest-even bfloat16 bits (uint16)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


class WarmStartNet:
    """Network state on the GPU: FP32 master weights, bfloat16 copies, Adam
    moments, activations and gradients for a fixed batch and grid."""

    def __init__(self, h, w, batch, seed=0):
        import torch
        self.torch = torch
        self.h, self.w, self.batch = h, w, batch
        self.dev = "cuda"
        self.stream = torch.cuda.current_stream().cuda_stream
        rng = np.random.default_rng(seed)
        self.W, self.b, self.Wb = [], [], []
        self.mW, self.vW, self.mb, self.vb = [], [], [], []
        self.gW, self.gb = [], []
        for li in range(5):
            cin, cout = CHANNELS[li], CHANNELS[li + 1]
            std = math.sqrt(1.0 / (9 * cin))
            w0 = rng.normal(scale=std, size=(cout, cin, 3, 3)).astype(np.float32)
            self.W.append(torch.tensor(w0, device=self.dev))
            self.b.append(torch.zeros(cout, dtype=torch.float32, device=self.dev))
            self.Wb.append(torch.empty((cout, cin, 3, 3), dtype=torch.int16, device=self.dev))
            for lst, t in ((self.mW, w0), (self.vW, w0), (self.gW, w0)):
                lst.append(torch.zeros(t.shape, dtype=torch.float32, device=self.dev))
            for lst in (self.mb, self.vb, self.gb):
                lst.append(torch.zeros(cout, dtype=torch.float32, device=self.dev))
            self._chk(B.lib().sc_nn_to_bf16(self.W[li].data_ptr(), self.Wb[li].data_ptr(), self.W[li].numel(),
                                            self.stream), "sc_nn_to_bf16")
        self.acts = [torch.empty((batch, c, h, w), dtype=torch.float32, device=self.dev) for c in CHANNELS]
        self.gact = [torch.empty((batch, c, h, w), dtype=torch.float32, device=self.dev) for c in CHANNELS]
        self.prm = torch.empty((batch, 4), dtype=torch.float32, device=self.dev)
        self.nblk_w = 512
        nsc = max(B.lib().sc_nn_bwd_weight_scratch_floats(CHANNELS[i], CHANNELS[i + 1], self.nblk_w)
                  for i in range(5))
        self.wscratch = torch.empty(nsc, dtype=torch.float32, device=self.dev)
        self.wt = torch.empty(32 * 32 * 9, dtype=torch.int16, device=self.dev)
        self.nblk_mse = 256
        self.mse_part = torch.empty(self.nblk_mse, dtype=torch.float64, device=self.dev)
        self.t = 0

    @staticmethod
    def _chk(rc, what):
        if rc != B.SC_OK:
            raise B.ScError(rc, what)

    # -------------------------------------------------------------- passes --
    def set_params(self, prm_rows):
        """prm_rows: [batch][4] normalised parameters (numpy, or a float32
        device tensor, which is then used without a host round trip)."""
        if isinstance(prm_rows, self.torch.Tensor):
            self.prm.copy_(prm_rows)
        else:
            self.prm.copy_(self.torch.tensor(np.asarray(prm_rows, dtype=np.float32), device=self.dev))
        self._chk(B.lib().sc_nn_features(self.prm.data_ptr(), self.acts[0].data_ptr(), self.batch, self.h, self.w,
                                         SCALE_R, self.stream), "sc_nn_features")

    def forward(self):
        """The five convolutions; the hidden layers' tanh is fused into the
        convolution's store."""
        L = B.lib()
        for li in range(5):
            cin, cout = CHANNELS[li], CHANNELS[li + 1]
            fn = L.sc_nn_conv3x3_fwd_tanh if li < 4 else L.sc_nn_conv3x3_fwd
            self._chk(fn(self.acts[li].data_ptr(), self.Wb[li].data_ptr(), self.b[li].data_ptr(),
                         self.acts[li + 1].data_ptr(), self.batch, cin, cout, self.h, self.w, self.stream),
                      "conv fwd")
        return self.acts[5]

    def loss_and_grad(self, target):
        """MSE against target [batch,1,h,w] (torch, device); fills the output
        gradient; returns the loss as a device-side partial vector."""
        self._chk(B.lib().sc_nn_mse(self.acts[5].data_ptr(), target.data_ptr(), self.gact[5].data_ptr(),
                                    self.mse_part.data_ptr(), self.nblk_mse, self.acts[5].numel(), self.stream),
                  "mse")
        return self.mse_part

    def backward(self):
        """Gradients of every layer.  The input gradient of layers 1..4 is
        multiplied by the tanh derivative of their input activation in the
        same pass (sc_nn_conv3x3_bwd_data_tanh), so gact[li] holds the
        gradient w.r.t. layer li's pre-activation when layer li - 1 uses it."""
        L = B.lib()
        for li in range(4, -1, -1):
            cin, cout = CHANNELS[li], CHANNELS[li + 1]
            g = self.gact[li + 1]
            self._chk(L.sc_nn_conv3x3_bwd_weight(self.acts[li].data_ptr(), g.data_ptr(), self.wscratch.data_ptr(),
                                                 self.nblk_w, self.gW[li].data_ptr(), self.gb[li].data_ptr(),
                                                 self.batch, cin, cout, self.h, self.w, self.stream), "bwd w")
            if li > 0:
                self._chk(L.sc_nn_conv3x3_bwd_data_tanh(g.data_ptr(), self.Wb[li].data_ptr(), self.wt.data_ptr(),
                                                        self.acts[li].data_ptr(), self.gact[li].data_ptr(),
                                                        self.batch, cin, cout, self.h, self.w, self.stream),
                          "bwd data")

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        L = B.lib()
        for li in range(5):
            self._chk(L.sc_nn_adam(self.W[li].data_ptr(), self.gW[li].data_ptr(), self.mW[li].data_ptr(),
                                   self.vW[li].data_ptr(), self.Wb[li].data_ptr(), self.W[li].numel(), lr, b1, b2,
                                   eps, self.t, self.stream), "adam W")
            self._chk(L.sc_nn_adam(self.b[li].data_ptr(), self.gb[li].data_ptr(), self.mb[li].data_ptr(),
                                   self.vb[li].data_ptr(), None, self.b[li].numel(), lr, b1, b2, eps, self.t,
                                   self.stream), "adam b")

    # ------------------------------------------------------------- helpers --
    def weights_numpy(self):
        """(bf16-rounded weights as float64, biases) per layer, for checks."""
        out = []
        for li in range(5):
            wb = self.Wb[li].cpu().numpy().view(np.uint16).astype(np.uint32) << 16
            out.append((wb.view(np.float32).astype(np.float64), self.b[li].cpu().numpy().astype(np.float64)))
        return out


def steady_states(items, tol=1e-9, max_steps=200000, obs_every=100, stream=None):
    """Run droplets (dicts with rho0, order, G, tau) to their steady state in
    one batched sweep; returns (fields, steps per item, converged_by, wall s)."""
    t0 = time.perf_counter()
    bt = B.Batch(items, stream=stream, obs_every=obs_every)
    bt.step(max_steps, tol=tol)
    fields, steps, by = [], [], []
    for k in range(len(items)):
        fields.append(bt.observe(k)["rho"])
        st, cb = bt.status(k)
        steps.append(st)
        by.append(cb)
    bt.close()
    return fields, steps, by, time.perf_counter() - t0


def train(net, inputs, targets, epochs=20, lr=2e-3, log=None, seed=0):
    """inputs: [N][4] normalised parameters; targets: [N][h][w] densities.

    The whole training set stays in device memory; each epoch's mini-batches
    are gathered there in a shuffled order, and the loss partials of every
    mini-batch are kept on the device and read back once per epoch, so the
    host never waits on the GPU inside an epoch."""
    torch = net.torch
    n = len(inputs)
    tgt_dev = torch.tensor(np.asarray(targets, dtype=np.float32)[:, None], device=net.dev)
    inp_dev = torch.tensor(np.asarray(inputs, dtype=np.float32), device=net.dev)
    nbat = n // net.batch
    loss_rows = torch.zeros((max(nbat, 1), net.nblk_mse), dtype=torch.float64, device=net.dev)
    tgt = torch.empty((net.batch, 1, net.h, net.w), dtype=torch.float32, device=net.dev)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = torch.tensor(rng.permutation(n)[:nbat * net.batch].reshape(nbat, net.batch), device=net.dev)
        for k in range(nbat):
            idx = order[k]
            net.set_params(inp_dev.index_select(0, idx))
            net.forward()
            torch.index_select(tgt_dev, 0, idx, out=tgt)
            part = net.loss_and_grad(tgt)
            net.backward()
            net.adam(lr=lr * (0.5 ** (ep // max(1, epochs // 3))))
            loss_rows[k].copy_(part)
        tot = float(loss_rows[:nbat].sum().item()) / (net.batch * net.h * net.w) if nbat else 0.0
        hist.append(tot / max(nbat, 1))
        if log:
            log("epoch %d loss %.3e" % (ep, hist[-1]))
    return hist


def predict(net, inputs):
    """Raw network outputs [N][h][w] (numpy float64, TARGET_SCALE x residual)
    for normalised parameter rows."""
    out = []
    n = len(inputs)
    for s in range(0, n, net.batch):
        rows = list(inputs[s:s + net.batch])
        k = len(rows)
        rows += [rows[-1]] * (net.batch - k)
        net.set_params(rows)
        y = net.forward()
        out.extend(y[:k, 0].cpu().numpy().astype(np.float64))
    return out


def start_fields(net, inputs, bases, masses):
    """Initial densities of the learned start (numpy float64 [N][h][w]):
    forward pass, then sc_nn_start_field (square-symmetry average of
    base + output / TARGET_SCALE, clamp to RHO_CLAMP, shift to the mass)."""
    torch = net.torch
    out = []
    n = len(inputs)
    for s in range(0, n, net.batch):
        rows = list(inputs[s:s + net.batch])
        k = len(rows)
        pad = net.batch - k
        rows += [rows[-1]] * pad
        net.set_params(rows)
        y = net.forward()
        b = list(bases[s:s + k]) + [bases[s + k - 1]] * pad
        m = list(masses[s:s + k]) + [masses[s + k - 1]] * pad
        bd = torch.tensor(np.stack(b), dtype=torch.float64, device=net.dev)
        md = torch.tensor(np.asarray(m, dtype=np.float64), device=net.dev)
        od = torch.empty_like(bd)
        net._chk(B.lib().sc_nn_start_field(y.data_ptr(), bd.data_ptr(), md.data_ptr(), od.data_ptr(), net.batch,
                                           net.h, net.w, 1.0 / TARGET_SCALE, RHO_CLAMP[0], RHO_CLAMP[1],
                                           net.stream), "sc_nn_start_field")
        out.extend(od[:k].cpu().numpy())
    return out


def make_dataset(n_train, n_test, side, tol, max_steps, obs_every, chunk, seed, jitter=False, log=print):
    """Steady states of the sweep's items (side fixed) from the tanh start
    (without the per-node jitter unless `jitter`)."""
    from workload import droplet_rho, sweep_items
    items = sweep_items(n_train + n_test, seed=seed, sides=side)
    fields, steps, conv = [], [], []
    t_gen = 0.0
    for s in range(0, len(items), chunk):
        part = [{"rho0": droplet_rho((side, side), it["R"], seed=it["seed"] if jitter else None),
                 "order": it["order"], "G": it["G"], "tau": it["tau"]} for it in items[s:s + chunk]]
        f, st, by, wall = steady_states(part, tol=tol, max_steps=max_steps, obs_every=obs_every)
        fields += f
        steps += st
        conv += by
        t_gen += wall
        log("steady states %d/%d (%.1f s)" % (min(s + chunk, len(items)), len(items), t_gen))
    return {"items": items, "fields": fields, "steps": steps, "conv": conv, "gen_wall_s": t_gen,
            "n_train": n_train, "side": side, "tol": tol, "max_steps": max_steps, "obs_every": obs_every,
            "jitter": jitter}


def _runs(starts, items, init, tol, max_steps, obs_every, precision="fp32"):
    """Batched runs of `items` from the densities `starts`."""
    run = [{"rho0": r, "order": it["order"], "G": it["G"], "tau": it["tau"], "init": init, "precision": precision}
           for r, it in zip(starts, items)]
    return steady_states(run, tol=tol, max_steps=max_steps, obs_every=obs_every)


def evaluate(ds, epochs=300, batch=16, lr=1e-3, fp64_baseline=8, seed=2026, tols=(1e-10,), log=print):
    """Train on the dataset's training items, then compare steps and wall
    time to steady state on its held-out items.  Starts (batched runs):
      tanh            the tanh start, f = feq(rho, 0) (the method without the net)
      tanh_rest       the tanh start at rest in the forced sense
      learned         the learned start at rest (inference included in its time)
      learned_eq      the learned start with f = feq(rho, 0)
    all with the FP64 state, where the steady-state rule is the literal
    max|u| change < tol; then tanh_fp32 and learned_fp32 with the FP32 state
    and its rules (sc_lbm_step), and plain per-droplet FP64 runs from the
    tanh start (first items), for each tolerance in `tols` (None = the
    dataset's)."""
    from workload import droplet_rho
    torch = __import__("torch")
    items, fields, conv = ds["items"], ds["fields"], ds["conv"]
    side, max_steps, obs_every = ds["side"], ds["max_steps"], ds["obs_every"]
    n_train = ds["n_train"]
    base = lambda it: droplet_rho((side, side), it["R"])  # noqa: E731  tanh start
    ok = [k for k in range(len(items)) if conv[k] > 0]
    train_idx = [k for k in ok if k < n_train]
    test_idx = [k for k in ok if k >= n_train]
    test_items = [items[k] for k in test_idx]
    inputs = [normalise(it["R"], it["G"], it["tau"], it["order"]) for it in items]
    resid = {k: TARGET_SCALE * (fields[k] - base(items[k])) for k in ok}
    net = WarmStartNet(side, side, batch, seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, [inputs[k] for k in train_idx], [resid[k] for k in train_idx], epochs=epochs, lr=lr,
                 log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    bases = [base(it) for it in test_items]
    t0 = time.perf_counter()
    starts = start_fields(net, [inputs[k] for k in test_idx], bases, [b.sum() for b in bases])
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    raw = [b + r / TARGET_SCALE for b, r in zip(bases, predict(net, [inputs[k] for k in test_idx]))]
    nt = max(1, len(test_idx))

    def rel(a, k):
        return float(np.max(np.abs(a - fields[k])) / np.max(fields[k]))

    def rms(a, k):
        return float(np.sqrt(np.mean((a - fields[k]) ** 2)))
    res = {
        "n_train": len(train_idx), "n_test": len(test_idx), "not_converged": int(sum(1 for c in conv if c <= 0)),
        "side": side, "dataset_tol": ds["tol"], "dataset_jitter": ds.get("jitter", True), "epochs": epochs,
        "lr": lr, "loss_first": hist[0], "loss_last": hist[-1], "gen_wall_s": ds["gen_wall_s"],
        "train_wall_s": t_train, "inference_wall_s": t_inf,
        "err_max_rel_median": {"tanh": float(np.median([rel(b, k) for b, k in zip(bases, test_idx)])),
                               "raw_prediction": float(np.median([rel(p, k) for p, k in zip(raw, test_idx)])),
                               "learned": float(np.median([rel(p, k) for p, k in zip(starts, test_idx)]))},
        "err_rms_median": {"tanh": float(np.median([rms(b, k) for b, k in zip(bases, test_idx)])),
                           "raw_prediction": float(np.median([rms(p, k) for p, k in zip(raw, test_idx)])),
                           "learned": float(np.median([rms(p, k) for p, k in zip(starts, test_idx)]))},
        "test_items": [{"R": float(it["R"]), "G": float(it["G"]), "tau": float(it["tau"]), "order": int(it["order"])}
                       for it in test_items],
        "runs": {},
    }
    for tol in tols:
        tol = ds["tol"] if tol is None else tol
        key = "%.0e" % tol
        out = {}
        for name, st, init, prec in (("tanh", bases, "equilibrium", "fp64"), ("tanh_rest", bases, "rest", "fp64"),
                                     ("learned", starts, "rest", "fp64"),
                                     ("learned_eq", starts, "equilibrium", "fp64"),
                                     ("tanh_fp32", bases, "equilibrium", "fp32"),
                                     ("learned_fp32", starts, "rest", "fp32")):
            f, steps, by, wall = _runs(st, test_items, init, tol, max_steps, obs_every, prec)
            extra = t_inf if name.startswith("learned") else 0.0
            out[name] = {"steps_mean": float(np.mean(steps)), "steps_median": float(np.median(steps)),
                         "wall_s_per_item": (wall + extra) / nt, "converged": int(sum(1 for v in by if v > 0)),
                         "quarantined": int(sum(1 for v in by if v < 0)), "fields": f, "steps": steps,
                         "converged_by": [int(v) for v in by]}
            log("%s tol %s: mean steps %.0f, %.4f s per droplet" % (name, key, out[name]["steps_mean"],
                                                                  out[name]["wall_s_per_item"]))
        for name in list(out):
            ref = out["tanh_fp32" if name.endswith("fp32") else "tanh"]["steps"]
            out[name]["steps_ratio_median_vs_tanh"] = float(np.median(np.array(out[name]["steps"]) /
                                                                      np.maximum(np.array(ref), 1)))
            out[name]["faster_than_tanh"] = int(np.sum(np.array(out[name]["steps"]) < np.array(ref)))
        agree = [float(np.max(np.abs(a - b))) for a, b in zip(out["learned"]["fields"], out["tanh"]["fields"])]
        out["steady_fields_max_abs_diff_median"] = float(np.median(agree)) if agree else None
        t0 = time.perf_counter()
        fp64_steps = []
        for it, b in list(zip(test_items, bases))[:fp64_baseline]:
            sim = B.Sim(b, "D2Q9", order=it["order"], G=it["G"], tau=it["tau"], precision="fp64",
                        obs_every=obs_every)
            rc, done = sim.step(max_steps, tol=tol)
            fp64_steps.append(done)
            sim.close()
        torch.cuda.synchronize()
        nb = max(1, min(fp64_baseline, len(test_idx)))
        out["fp64"] = {"steps_mean": float(np.mean(fp64_steps)) if fp64_steps else None,
                       "wall_s_per_item": (time.perf_counter() - t0) / nb, "items": nb}
        for name in out:
            if isinstance(out[name], dict) and "steps" in out[name]:
                out[name].pop("fields", None)
                out[name]["steps"] = [int(v) for v in out[name]["steps"]]
        res["runs"][key] = out
    return res


def run_experiment(n_train=2000, n_test=200, side=256, tol=1e-8, epochs=300, batch=16, lr=1e-3,
                   max_steps=150000, obs_every=200, chunk=64, fp64_baseline=8, seed=2026, jitter=False,
                   tols=(1e-10,), log=print):
    """The 256^2 warm-start experiment: dataset from batched sweeps, then evaluate()."""
    ds = make_dataset(n_train, n_test, side, tol, max_steps, obs_every, chunk, seed, jitter=jitter, log=log)
    return evaluate(ds, epochs=epochs, batch=batch, lr=lr, fp64_baseline=fp64_baseline, seed=seed, tols=tols,
                    log=log)


def time_training(n=512, side=256, batch=16, epochs=3, seed=0):
    """Wall time of training epochs on synthetic tanh-profile targets (the
    network kernels at the experiment's sizes, without the LBM dataset):
    returns seconds per epoch and per item."""
    import torch
    rng = np.random.default_rng(seed)
    inputs = [normalise(rng.uniform(8, 85), rng.uniform(-5.5, -4.5), 1.0, 8) for _ in range(n)]
    yy, xx = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    r = np.sqrt((xx - side // 2) ** 2 + (yy - side // 2) ** 2)
    targets = [np.tanh((r - rng.uniform(8, 85)) / 3.0).astype(np.float32) for _ in range(n)]
    net = WarmStartNet(side, side, batch, seed=seed + 1)
    train(net, inputs[:2 * batch], targets[:2 * batch], epochs=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, inputs, targets, epochs=epochs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / epochs
    return {"items": n, "side": side, "batch": batch, "epochs": epochs, "s_per_epoch": dt,
            "ms_per_item_epoch": dt / n * 1e3, "loss": hist}


if __name__ == "__main__":
    import argparse
    import json
    import os
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="learned warm start experiment (droplet sweep on side^2 grids)")
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=200)
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-8, help="steady-state rule of the dataset runs")
    ap.add_argument("--eval-tols", default="1e-10", help="rules the starts are compared at")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--jitter", action="store_true", help="dataset runs from the jittered tanh start")
    ap.add_argument("--out", default=None)
    ap.add_argument("--time-training", action="store_true",
                    help="only time training epochs on synthetic targets (the network kernels)")
    a = ap.parse_args()
    if a.time_training:
        print(json.dumps(time_training(side=a.side)), flush=True)
        sys.exit(0)
    res = run_experiment(n_train=a.n_train, n_test=a.n_test, side=a.side, tol=a.tol, epochs=a.epochs, lr=a.lr,
                         jitter=a.jitter, tols=tuple(float(t) for t in a.eval_tols.split(",")),
                         log=lambda m: print(m, flush=True))
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
