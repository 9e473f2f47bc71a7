"""Learned warm start for droplet runs (an addition to the paper's method).

A five-layer 3x3 convolutional net (5 -> 32 -> 32 -> 32 -> 32 -> 1 channels,
tanh between layers, circular padding, bfloat16 weights with FP32
accumulation) maps the droplet parameters (R, G, tau, stencil order,
broadcast as channels) plus the radial coordinate grid to the steady density
field.  Its prediction, shifted to the mass of the usual tanh start (mass is
conserved by the step, so the steady state is fixed by it), replaces the
tanh profile as the initial condition; the lattice Boltzmann iteration still
runs to its own steady state and remains the judge of it.

Every arithmetic step runs in the library's kernels (sc_nn_* for the net,
sc_lbm_batch_* for the data); torch only allocates device memory and
provides the stream.  There is no CPU fallback.
"""
import math
import time

import numpy as np

from . import sc_lbm as B

CHANNELS = [5, 32, 32, 32, 32, 1]
SCALE_R = 100.0


def normalise(R, G, tau, order):
    """Parameters as the net sees them (roughly unit range)."""
    return [R / 100.0, (G + 5.0) / 0.5, (tau - 1.0) / 0.2, (order - 7.0) / 3.0]


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
    """Shift the prediction uniformly to the mass of rho_ref."""
    return rho_pred + (rho_ref.sum() - rho_pred.sum()) / rho_pred.size
