"""GPU parity of the start at rest in the forced sense (SC_INIT_REST:
f = feq(rho0, -F / (2 rho0)), so that (sum f c + F/2) / rho = 0 at t = 0)
against the FP64 oracle, on every lattice and kernel family, single domains
and the batched sweep.

Tolerances as for the other parity tests: FP64 state <= 1e-11 pointwise;
FP32 state density <= 1e-5 relative, velocity <= 1e-3 of max |u| plus the
FP32 momentum resolution (1e-7 max rho).  At t = 0, where the oracle's
velocity is zero, the GPU's is bounded by the resolution of the first
moment of the stored state divided by the density: the shifted values
g_b = f_b - w_b rho_ref are at most w_b max(1, |rho - rho_ref|) in size
and each is rounded to u_r = 2^-24 (2^-53 for the FP64 state) of it, so
|u| <= u_r sum_b |c_b| w_b max(1, |rho - rho_ref|) / min rho, taken with
a factor 4 for the sums (about 1e-6 here in FP32)."""
import warnings

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_helpers import pre_collision_from_state, rel_err, say
from workload import droplet_rho

pytestmark = pytest.mark.gpu
warnings.simplefilter("ignore")

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1906_11027_amd import Batch, Sim  # noqa: E402

TOL = {"fp32": (1e-5, 1e-3), "fp64": (1e-11, 1e-9)}
UFLOOR = {"fp32": 1e-7, "fp64": 1e-15}

CASES = [
    ("D2Q9", (70, 45), dict(order=8, G=-5.0, tau=1.0)),
    ("D2Q9", (66, 40), dict(order=6, G=-5.0, tau=0.8, forcing="edm")),
    ("D2Q13", (60, 41), dict(order=6, G=-6.0, tau=0.9, forcing="edm")),
    ("D2Q25", (58, 43), dict(order=8, G=-5.0 * 12 / 7, tau=1.0)),
    ("D3Q19", (20, 18, 17), dict(order=8, G=-5.0, tau=1.0, collision="mrt")),
]


def _compare(sim, orc, prec, label):
    got = sim.observe()
    ref = orc.fields()
    er = rel_err(got["rho"], ref["rho"])
    umax = max(np.max(np.abs(ref["u"])), 1e-12)
    du = float(np.max(np.abs(got["u"] - ref["u"])))
    say("%s: rho rel err %.3e, u err %.3e (max|u| %.3e)" % (label, er, du, umax))
    tr, tu = TOL[prec]
    assert er <= tr, (label, er)
    assert du <= tu * umax + UFLOOR[prec] * float(np.max(ref["rho"])), (label, du / umax)
    return got


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("lattice,shape,kw", CASES)
def test_rest_start_parity(lattice, shape, kw, prec):
    say("case rest start", lattice, shape, kw, prec)
    rho0 = droplet_rho(shape, min(shape) / 4.0, seed=5)
    sim = Sim(rho0, lattice, precision=prec, init="rest", **kw)
    orc = O.Oracle(rho0, lattice, init="rest", **kw)
    got = sim.observe()
    ref = orc.fields()
    assert np.max(np.abs(ref["u"])) < 1e-15
    er = rel_err(got["rho"], ref["rho"])
    u0 = float(np.max(np.abs(got["u"])))
    _, c, w, _ = O.lattice_table(lattice)
    cw = float((np.sqrt((c * c).sum(axis=1)) * w).sum())
    big = max(1.0, float(np.max(np.abs(rho0 - sim.rho_ref))))
    unit = 2.0 ** -24 if prec == "fp32" else 2.0 ** -53
    floor = 4 * unit * cw * big / float(np.min(rho0))
    say("%s %s t=0: rho rel err %.3e, max|u| %.3e (bound %.3e)" % (lattice, prec, er, u0, floor))
    assert er <= TOL[prec][0]
    assert u0 <= floor
    if prec == "fp64":
        f = pre_collision_from_state(sim, O.lattice_table(lattice)[1])
        assert np.max(np.abs(f - orc.get_f())) < 1e-14
    for st in (1, 49):
        sim.step(st)
        orc.step(st)
        _compare(sim, orc, prec, "%s %s t=%d" % (lattice, prec, orc.steps))
    sim.close()


def test_rest_start_every_d2q9_variant():
    """The initial state does not depend on the launch shape: every D2Q9
    shape (one- and two-step) steps the same rest start to the oracle."""
    from paper_1906_11027_amd import sc_lbm as B
    rho0 = droplet_rho((67, 53), 14, seed=6)
    kw = dict(order=8, G=-5.0, tau=1.0)
    orc = O.Oracle(rho0, "D2Q9", init="rest", **kw).step(20)
    for v in range(B.sc_lbm_num_variants(B.make_params("D2Q9"))):
        sim = Sim(rho0, "D2Q9", variant=v, precision="fp64", init="rest", **kw)
        sim.step(20)
        _compare(sim, orc, "fp64", "variant %s" % sim.variant)
        sim.close()


def test_batched_rest_start_parity():
    items = []
    for side, R, G, tau, order in [(64, 14, -5.0, 1.0, 8), (96, 20, -4.8, 0.8, 4),
                                   (80, 18, -5.3, 1.2, 10)]:
        items.append({"rho0": droplet_rho((side, side), R), "order": order, "G": G, "tau": tau,
                      "precision": "fp64", "init": "rest"})
    bt = Batch(items)
    bt.step(30)
    for k, it in enumerate(items):
        kw = {key: it[key] for key in ("order", "G", "tau")}
        orc = O.Oracle(it["rho0"], "D2Q9", init="rest", **kw).step(30)
        got = bt.observe(k)
        ref = orc.fields()
        assert rel_err(got["rho"], ref["rho"]) < 1e-11
        assert np.max(np.abs(got["u"] - ref["u"])) < 1e-9 * np.max(np.abs(ref["u"])) + 1e-15
    bt.close()
