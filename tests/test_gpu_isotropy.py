"""The 256^2 droplet of the isotropy study (D2Q9 SRT, psi = 1 - exp(-rho),
G = -5, tau = 1, R = 40, seeded tanh start) against the FP64 oracle's own
runs of it, stored by tests/golden/make_droplet_256_orders.py: E4, E6, E8
and E10 for 50,000 steps each (Sec. 2, 3).

FP64 state: every stored checkpoint's observables within 1e-9 relative
(Laplace jump: 1e-9 of p_in), and the final density and velocity along the
row and the column through the centre within 2e-10 absolute.  At 10^4 steps
the FP64 GPU state stays within 1e-11 of the oracle; the summation order
differs per step at round-off (2^-53), and the bound allows that to grow
linearly over 5 x 10^4 steps with a factor 4 to spare.

FP32 state (the default storage shift), at the final checkpoint:
- the |u| norms within 1e-3 relative, the Laplace jump within 1e-4 and the
  density extremes within 1e-5 relative (the stated FP32 tolerances);
- along the centre row and column, the density within 1e-5 relative at
  bulk nodes (where the oracle's profile changes by less than 1e-4 per
  node);
- the interface crossings along those lines (where rho passes the mean of
  the extremes) within 5e-3 nodes of the oracle's, and every node within
  3e-3 absolute in density.
Round-off moves the interface of the FP32 run slightly over 5 x 10^4 steps,
because the droplet's position and shape are neutral or slow modes. The
density error at interface nodes is that shift times the slope (at most
about 0.5 per node).  The shift is largest for E4, whose jitter-seeded
shape mode is still evolving at 5 x 10^4 steps: 2.3e-3 nodes, against
2.5e-4 for E8."""
import json
import os

import numpy as np
import pytest

from paper_1906_11027_amd import Sim
from tests.gpu_helpers import say
from workload import droplet_rho

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "droplet_256_orders_oracle.json")
with open(GOLD_PATH) as _fh:
    GOLD = json.load(_fh)
ORDERS = sorted(GOLD["orders"], key=int)
OBS = ("max_u", "mean_u", "l2_u", "rho_in", "rho_out", "rho_min", "rho_max", "mass", "radius")


def _rho0():
    return droplet_rho(tuple(GOLD["shape"]), GOLD["R"], seed=GOLD["seed"])


def _lines(out, g):
    cy, cx = g["row_y"], g["col_x"]
    return {"rho_row": out["rho"][:, cy], "ux_row": out["u"][0][:, cy], "uy_row": out["u"][1][:, cy],
            "rho_col": out["rho"][cx, :], "ux_col": out["u"][0][cx, :], "uy_col": out["u"][1][cx, :]}


@pytest.mark.parametrize("order", ORDERS)
def test_fp64_matches_oracle_run(order):
    g = GOLD["orders"][order]
    say("case droplet 256 E%s fp64, %d steps" % (order, g["steps"]))
    sim = Sim(_rho0(), "D2Q9", order=int(order), G=GOLD["G"], tau=GOLD["tau"], precision="fp64",
              obs_every=g["every"])
    worst = 0.0
    for ref in g["traj"]:
        sim.step(g["every"])
        ob = sim.observe(fields=False)["obs"]
        assert ob["step"] == ref["step"]
        for k in OBS:
            e = abs(ob[k] - ref[k]) / abs(ref[k])
            worst = max(worst, e)
            assert e <= 1e-9, (ref["step"], k, ob[k], ref[k])
        assert abs(ob["dp"] - ref["dp"]) <= 1e-9 * abs(ref["p_in"]), (ref["step"], ob["dp"], ref["dp"])
    got = _lines(sim.observe(), g)
    sim.close()
    errs = {k: float(np.max(np.abs(v - np.asarray(g[k])))) for k, v in got.items()}
    say("E%s fp64: worst observable rel err %.2e; centre lines %s" % (
        order, worst, " ".join("%s %.1e" % kv for kv in errs.items())))
    for k, e in errs.items():
        assert e <= 2e-10, (k, e)


@pytest.mark.parametrize("order", ORDERS)
def test_fp32_matches_oracle_run(order):
    g = GOLD["orders"][order]
    say("case droplet 256 E%s fp32, %d steps" % (order, g["steps"]))
    # one fixed launch shape (tile32x8r1, the small-grid default): an FP32 run's
    # rounding, and so its far-field noise, depends on the shape, and an
    # autotuning call earlier in the process may change the default; every
    # shape's agreement with this one is checked in test_gpu_parity
    sim = Sim(_rho0(), "D2Q9", order=int(order), G=GOLD["G"], tau=GOLD["tau"], obs_every=g["every"], variant=2)
    assert sim.variant == "tile32x8r1"
    sim.step(g["steps"])
    out = sim.observe()
    ob, ref = out["obs"], g["traj"][-1]
    shift = sim.rho_ref
    sim.close()
    assert ob["step"] == ref["step"]
    rel = {k: abs(ob[k] - ref[k]) / abs(ref[k]) for k in ("max_u", "mean_u", "l2_u", "dp", "rho_min", "rho_max")}
    got = _lines(out, g)
    rho_v, rho_l = ref["rho_min"], ref["rho_max"]
    mid = 0.5 * (rho_v + rho_l)
    line_err = {}
    for k in ("rho_row", "rho_col"):
        r = np.asarray(g[k])
        slope = 0.5 * np.abs(np.roll(r, -1) - np.roll(r, 1))
        bulk = slope < 1e-4
        d = np.abs(got[k] - r)
        xr, xg = _crossings(r, mid), _crossings(got[k], mid)
        assert len(xr) == len(xg) == 2, (k, xr, xg)
        assert bulk.sum() > r.size // 2, (k, int(bulk.sum()))
        line_err[k] = (float(np.max(d[bulk] / r[bulk])), float(np.max(d)), float(np.max(np.abs(xg - xr))))
    say("E%s fp32 (shift %.4f): %s; centre lines (bulk rel, any abs, crossing shift) %s" % (
        order, shift, " ".join("%s %.1e" % kv for kv in rel.items()), line_err))
    for k in ("max_u", "mean_u", "l2_u"):
        assert rel[k] <= 1e-3, (k, rel[k])
    assert rel["dp"] <= 1e-4
    assert rel["rho_min"] <= 1e-5 and rel["rho_max"] <= 1e-5
    for k, (bulk_rel, any_abs, shift_nodes) in line_err.items():
        assert bulk_rel <= 1e-5, (k, bulk_rel)
        assert shift_nodes <= 5e-3, (k, shift_nodes)
        assert any_abs <= 3e-3, (k, any_abs)


def _crossings(v, level):
    """Positions (linear interpolation) where the line crosses `level`."""
    v = np.asarray(v, dtype=np.float64) - level
    i = np.nonzero(np.sign(v[:-1]) != np.sign(v[1:]))[0]
    return np.array([j + v[j] / (v[j] - v[j + 1]) for j in i])
