"""Learned warm start for droplet runs (an addition to the paper's method).

A five-layer 3x3 convolutional net (5 -> 32 -> 32 -> 32 -> 32 -> 1 channels,
tanh between layers, circular padding, bfloat16 weights with FP32
accumulation) maps the droplet parameters (R, G, tau, stencil order,
broadcast as channels) plus the radial coordinate grid to the steady density
field.  It is trained on the residual between the steady field and the usual
tanh start (scaled by TARGET_SCALE), so an untrained net reproduces the tanh
start and training moves it towards the steady state.  The prediction
(tanh start + residual), clamped to a physical range and shifted to the mass
of the tanh start (mass is conserved by the step, so the steady state is
fixed by it), becomes the initial condition; the lattice Boltzmann iteration
still runs to its own steady state and alone decides when it is reached.

Every arithmetic step runs in the library's kernels (sc_nn_* for the net,
sc_lbm_batch_* for the data); torch only allocates device memory and
provides the stream.  There is no CPU fallback.
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
        self.nblk_w = 128
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
        """prm_rows: [batch][4] normalised parameters (numpy)."""
        t = self.torch.tensor(np.asarray(prm_rows, dtype=np.float32), device=self.dev)
        self.prm.copy_(t)
        self._chk(B.lib().sc_nn_features(self.prm.data_ptr(), self.acts[0].data_ptr(), self.batch, self.h, self.w,
                                         SCALE_R, self.stream), "sc_nn_features")

    def forward(self):
        L = B.lib()
        for li in range(5):
            cin, cout = CHANNELS[li], CHANNELS[li + 1]
            self._chk(L.sc_nn_conv3x3_fwd(self.acts[li].data_ptr(), self.Wb[li].data_ptr(), self.b[li].data_ptr(),
                                          self.acts[li + 1].data_ptr(), self.batch, cin, cout, self.h, self.w,
                                          self.stream), "conv fwd")
            if li < 4:
                self._chk(L.sc_nn_tanh_fwd(self.acts[li + 1].data_ptr(), self.acts[li + 1].numel(), self.stream),
                          "tanh fwd")
        return self.acts[5]

    def loss_and_grad(self, target):
        """MSE against target [batch,1,h,w] (torch, device); fills the output
        gradient; returns the loss as a device-side partial vector."""
        self._chk(B.lib().sc_nn_mse(self.acts[5].data_ptr(), target.data_ptr(), self.gact[5].data_ptr(),
                                    self.mse_part.data_ptr(), self.nblk_mse, self.acts[5].numel(), self.stream),
                  "mse")
        return self.mse_part

    def backward(self):
        L = B.lib()
        for li in range(4, -1, -1):
            cin, cout = CHANNELS[li], CHANNELS[li + 1]
            g = self.gact[li + 1]
            if li < 4:
                self._chk(L.sc_nn_tanh_bwd(self.acts[li + 1].data_ptr(), g.data_ptr(), g.numel(), self.stream),
                          "tanh bwd")
            self._chk(L.sc_nn_conv3x3_bwd_weight(self.acts[li].data_ptr(), g.data_ptr(), self.wscratch.data_ptr(),
                                                 self.nblk_w, self.gW[li].data_ptr(), self.gb[li].data_ptr(),
                                                 self.batch, cin, cout, self.h, self.w, self.stream), "bwd w")
            if li > 0:
                self._chk(L.sc_nn_conv3x3_bwd_data(g.data_ptr(), self.Wb[li].data_ptr(), self.wt.data_ptr(),
                                                   self.gact[li].data_ptr(), self.batch, cin, cout, self.h, self.w,
                                                   self.stream), "bwd data")

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
    """inputs: [N][4] normalised parameters; targets: [N][h][w] densities."""
    torch = net.torch
    n = len(inputs)
    tgt_host = np.asarray(targets, dtype=np.float32)[:, None]
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot = 0.0
        nb = 0
        for s in range(0, n - net.batch + 1, net.batch):
            idx = order[s:s + net.batch]
            net.set_params(np.asarray(inputs)[idx])
            net.forward()
            tgt = torch.tensor(np.ascontiguousarray(tgt_host[idx]), device=net.dev)
            part = net.loss_and_grad(tgt)
            net.backward()
            net.adam(lr=lr * (0.5 ** (ep // max(1, epochs // 3))))
            tot += float(part.cpu().numpy().sum()) / (net.batch * net.h * net.w)
            nb += 1
        hist.append(tot / max(nb, 1))
        if log:
            log("epoch %d loss %.3e" % (ep, hist[-1]))
    return hist


def predict(net, inputs):
    """Densities [N][h][w] (numpy float64) for normalised parameter rows."""
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


def mass_project(rho_pred, rho_ref):
    """Clamp the prediction to a physical density range, then shift it
    uniformly to the mass of rho_ref."""
    r = np.clip(rho_pred, RHO_CLAMP[0], RHO_CLAMP[1])
    return r + (rho_ref.sum() - r.sum()) / r.size


def make_dataset(n_train, n_test, side, tol, max_steps, obs_every, chunk, seed, log=print):
    """Steady states of the sweep's items (side fixed) from the tanh start."""
    from workload import droplet_rho, sweep_items
    items = sweep_items(n_train + n_test, seed=seed, sides=side)
    fields, steps, conv = [], [], []
    t_gen = 0.0
    for s in range(0, len(items), chunk):
        part = [{"rho0": droplet_rho((side, side), it["R"], seed=it["seed"]), "order": it["order"], "G": it["G"],
                 "tau": it["tau"]} for it in items[s:s + chunk]]
        f, st, by, wall = steady_states(part, tol=tol, max_steps=max_steps, obs_every=obs_every)
        fields += f
        steps += st
        conv += by
        t_gen += wall
        log("steady states %d/%d (%.1f s)" % (min(s + chunk, len(items)), len(items), t_gen))
    return {"items": items, "fields": fields, "steps": steps, "conv": conv, "gen_wall_s": t_gen,
            "n_train": n_train, "side": side, "tol": tol, "max_steps": max_steps, "obs_every": obs_every}


def evaluate(ds, epochs=20, batch=16, lr=2e-3, fp64_baseline=8, seed=2026, log=print):
    """Train on the dataset's training items, then compare steps and wall time
    to steady state on its held-out items: tanh start (batched FP32), learned
    start (batched FP32, inference included), plain per-droplet FP64 runs."""
    from workload import droplet_rho
    torch = __import__("torch")
    items, fields, conv = ds["items"], ds["fields"], ds["conv"]
    side, tol, max_steps, obs_every = ds["side"], ds["tol"], ds["max_steps"], ds["obs_every"]
    n_train = ds["n_train"]
    rho0 = lambda it: droplet_rho((side, side), it["R"], seed=it["seed"])  # noqa: E731
    base = lambda it: droplet_rho((side, side), it["R"])  # noqa: E731  tanh start without jitter
    ok = [k for k in range(len(items)) if conv[k] > 0]
    train_idx = [k for k in ok if k < n_train]
    test_idx = [k for k in ok if k >= n_train]
    inputs = [normalise(it["R"], it["G"], it["tau"], it["order"]) for it in items]
    resid = {k: TARGET_SCALE * (fields[k] - base(items[k])) for k in ok}
    net = WarmStartNet(side, side, batch, seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, [inputs[k] for k in train_idx], [resid[k] for k in train_idx], epochs=epochs, lr=lr,
                 log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    pred = [base(items[k]) + r / TARGET_SCALE
            for k, r in zip(test_idx, predict(net, [inputs[k] for k in test_idx]))]
    warm_items = [{"rho0": mass_project(p, rho0(items[k])), "order": items[k]["order"], "G": items[k]["G"],
                   "tau": items[k]["tau"]} for k, p in zip(test_idx, pred)]
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    wf, wst, wby, t_warm = steady_states(warm_items, tol=tol, max_steps=max_steps, obs_every=obs_every)
    cold_items = [{"rho0": rho0(items[k]), "order": items[k]["order"], "G": items[k]["G"],
                   "tau": items[k]["tau"]} for k in test_idx]
    cf, cst, cby, t_cold = steady_states(cold_items, tol=tol, max_steps=max_steps, obs_every=obs_every)
    t0 = time.perf_counter()
    fp64_steps = []
    for k in test_idx[:fp64_baseline]:
        it = items[k]
        sim = B.Sim(rho0(it), "D2Q9", order=it["order"], G=it["G"], tau=it["tau"], precision="fp64",
                    obs_every=obs_every)
        rc, done = sim.step(max_steps, tol=tol)
        fp64_steps.append(done)
        sim.close()
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    nb = max(1, min(fp64_baseline, len(test_idx)))
    nt = max(1, len(test_idx))
    pred_err = [float(np.max(np.abs(p - fields[k])) / np.max(fields[k])) for k, p in zip(test_idx, pred)]
    tanh_err = [float(np.max(np.abs(base(items[k]) - fields[k])) / np.max(fields[k])) for k in test_idx]
    agree = [float(np.max(np.abs(a - b))) for a, b, x, y in zip(wf, cf, wby, cby) if x > 0 and y > 0]
    return {
        "n_train": len(train_idx), "n_test": len(test_idx), "diverged": int(sum(1 for c in conv if c < 0)),
        "side": side, "tol": tol, "epochs": epochs, "lr": lr, "loss_first": hist[0], "loss_last": hist[-1],
        "gen_wall_s": ds["gen_wall_s"], "train_wall_s": t_train, "inference_wall_s": t_inf,
        "pred_max_rel_err_median": float(np.median(pred_err)),
        "tanh_max_rel_err_median": float(np.median(tanh_err)),
        "steps_tanh_mean": float(np.mean(cst)), "steps_warm_mean": float(np.mean(wst)),
        "steps_ratio_median": float(np.median(np.array(wst) / np.maximum(np.array(cst), 1))),
        "wall_tanh_batched_s_per_item": t_cold / nt,
        "wall_warm_batched_s_per_item": (t_warm + t_inf) / nt,
        "wall_fp64_per_droplet_s_per_item": t_fp64 / nb,
        "fp64_steps_mean": float(np.mean(fp64_steps)) if fp64_steps else None,
        "steady_fields_max_abs_diff_median": float(np.median(agree)) if agree else None,
        "warm_converged": int(sum(1 for v in wby if v > 0)),
    }


def run_experiment(n_train=2000, n_test=64, side=256, tol=1e-8, epochs=20, batch=16, lr=2e-3,
                   max_steps=150000, obs_every=200, chunk=64, fp64_baseline=8, seed=2026, log=print):
    """The 256^2 warm-start experiment: dataset from batched sweeps, then evaluate()."""
    ds = make_dataset(n_train, n_test, side, tol, max_steps, obs_every, chunk, seed, log=log)
    return evaluate(ds, epochs=epochs, batch=batch, lr=lr, fp64_baseline=fp64_baseline, seed=seed, log=log)


if __name__ == "__main__":
    import argparse
    import json
    import os
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="learned warm start experiment (droplet sweep on side^2 grids)")
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=64)
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = run_experiment(n_train=a.n_train, n_test=a.n_test, side=a.side, tol=a.tol, epochs=a.epochs, lr=a.lr,
                         log=lambda m: print(m, flush=True))
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
