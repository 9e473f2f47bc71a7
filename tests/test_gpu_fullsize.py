"""Parity at the full sizes the bench times, in the launch shape it times
(the autotuned one), on sampled boxes the oracle can compute.

Each bench workload -- 256^2 and 8192^2 D2Q9 E8, 128^3 and 320^3 D3Q19 MRT
E8, 8192^2 D2Q13 E6 and D2Q25 E8 with Peng-Robinson psi and EDM, and the
8192^2 D2Q9 and 320^3 D3Q19 runs of the FP64 state -- is
created as bench.py creates it, advanced a few launches from its droplet
start, and its state copied to the host.  For boxes placed across the
interface, in the bulk and across the periodic seams, the oracle restarts
from that state on the box (periodic on the box) and takes as many steps
as one launch advances.  The node values inside the box at a distance of
k (max|c| + R) + R from its faces depend only on data inside the box
(k steps of pull distance max|c| and force reach R, then the force of the
final fields), so there the oracle's FP64 result is the exact reference
for the GPU's launch.  Tolerances: those of the other parity tests (FP32:
density 1e-5 relative, velocity 1e-3 of the box's max|u| plus the FP32
momentum resolution 1e-7 max rho; FP64: 1e-11 and 1e-9).

The batched sweep runs at full size too (all 64 droplets of the sweep,
sides 64..512): four items, the largest and the smallest grid among them,
against whole-grid oracle runs from the same start."""
import numpy as np
import pytest

import bench
from oracle import oracle as O
from paper_1906_11027_amd import Batch, Sim
from paper_1906_11027_amd import sc_lbm as B
from tests.gpu_helpers import pre_collision_patch, rel_err, say
from workload import droplet_rho, sweep_items

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _boxes(shape, R_drop, size):
    """Boxes across the droplet's interface (+x and +y/+z sides), at the
    droplet centre and across the periodic corner."""
    dim = len(shape)
    ctr = [s // 2 for s in shape]
    half = [b // 2 for b in size]
    out = []
    for axis in (0, 1):
        lo = [ctr[d] - half[d] for d in range(dim)]
        lo[axis] = ctr[axis] + int(R_drop) - half[axis]
        out.append(tuple(lo))
    out.append(tuple(ctr[d] - half[d] for d in range(dim)))
    out.append(tuple(-half[d] for d in range(dim)))
    return out


@pytest.mark.parametrize("name", ["d2q9_e8_256", "d2q9_e8_8192", "d3q19_mrt_e8_128", "d3q19_mrt_e8_320",
                                  "d2q13_e6_pr_edm_8192", "d2q25_e8_pr_edm_8192", "d2q9_e8_8192_fp64",
                                  "d3q19_mrt_e8_320_fp64"])
def test_bench_workload_sampled_boxes(name):
    w = bench.WORKLOADS[name]
    kw, rho0 = bench.sim_kwargs(w)
    prec = w.get("precision", "fp32")
    tr, tu, floor = (1e-5, 1e-3, 1e-7) if prec == "fp32" else (1e-11, 1e-9, 1e-15)
    say("case full-size %s %s" % (name, w["shape"]))
    nodes = int(np.prod(w["shape"]))
    B.sc_lbm_autotune(B.make_params(w["lattice"], w["shape"], precision=prec, **kw),
                      steps=256 if nodes < 1 << 20 else 32)
    sim = Sim(rho0, w["lattice"], precision=prec, **kw)
    del rho0
    k = sim.steps_per_launch
    sim.step(8 * k)
    s0 = sim.state()
    sim.step(k)
    got = sim.observe()
    dim = sim.dim
    _, oc, _, _ = O.lattice_table(w["lattice"])
    reach = int(np.max(np.abs(np.asarray(O.stencil_table(dim, w["order"])[0]))))
    margin = k * (int(np.max(np.abs(oc))) + reach) + reach
    size = (48, 48) if dim == 2 else (20, 20, 20)
    okw = {key: v for key, v in kw.items()}
    for lo in _boxes(w["shape"], w["R"], size):
        f = pre_collision_patch(s0, sim, lo, size, oc)
        orc = O.Oracle(np.ones(size), w["lattice"], **okw)
        orc.set_f(f)
        orc.step(k)
        ref = orc.fields()
        inner = tuple(slice(margin, size[d] - margin) for d in range(dim))
        idx = np.ix_(*[np.arange(lo[d] + margin, lo[d] + size[d] - margin) % w["shape"][d] for d in range(dim)])
        g_rho, g_u = got["rho"][idx], got["u"][(slice(None),) + idx]
        r_rho, r_u = ref["rho"][inner], ref["u"][(slice(None),) + inner]
        er = rel_err(g_rho, r_rho)
        umax = max(float(np.max(np.abs(r_u))), 1e-12)
        du = float(np.max(np.abs(g_u - r_u)))
        say("%s %s box at %s (%d nodes inside): rho rel err %.2e, u err %.2e (box max|u| %.2e)" % (
            name, sim.variant, lo, r_rho.size, er, du, umax))
        assert er <= tr, (lo, er)
        assert du <= tu * umax + floor * float(np.max(r_rho)), (lo, du, umax)
    sim.close()


def test_batched_sweep_full_size():
    its = sweep_items(64, seed=1906)
    items = [{"rho0": droplet_rho((it["side"],) * 2, it["R"], seed=it["seed"]), "order": it["order"],
              "G": it["G"], "tau": it["tau"]} for it in its]
    say("case full-size batch: %d items, %d nodes" % (len(items), sum(it["rho0"].size for it in items)))
    bt = Batch(items)
    bt.step(20)
    sides = [it["side"] for it in its]
    pick = sorted({int(np.argmax(sides)), int(np.argmin(sides)),
                   next(i for i, it in enumerate(its) if it["order"] == 10),
                   next(i for i, it in enumerate(its) if it["tau"] == 0.8)})
    for i in pick:
        it = items[i]
        orc = O.Oracle(it["rho0"], "D2Q9", order=it["order"], G=it["G"], tau=it["tau"]).step(20)
        got, ref = bt.observe(i), orc.fields()
        er = rel_err(got["rho"], ref["rho"])
        umax = max(float(np.max(np.abs(ref["u"]))), 1e-12)
        du = float(np.max(np.abs(got["u"] - ref["u"])))
        say("batch item %d (side %d, E%d, tau %.1f): rho rel err %.2e, u err %.2e (max|u| %.2e)" % (
            i, sides[i], it["order"], it["tau"], er, du, umax))
        assert er <= 1e-5, (i, er)
        assert du <= 1e-3 * umax + 1e-7 * float(np.max(ref["rho"])), (i, du, umax)
    bt.close()
