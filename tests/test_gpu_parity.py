"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances.  FP32 state: density <= 1e-5 relative pointwise and velocity
<= 1e-3 of max |u| (plus the FP32 momentum resolution, 1e-7 max rho, where
max |u| is itself near round-off) up to 1,000 steps on the 64^2 droplet.
With the default storage shift (the median density) the density error
grows from ~1e-6 after one step to 1-7e-6 at 1,000 steps and ~9e-6 at
2,000 (interface nodes: the interface position responds to the rounding),
so longer runs are compared on the observables the method reports
(spurious max / mean |u| within 1e-3 relative, Laplace jump within 1e-4).
FP64 state: <= 1e-11 pointwise at any horizon tested.  Launch shapes agree
to rounding (<= 1e-6 FP32, 1e-14 FP64): every node's arithmetic is the
same, but the compiler contracts multiply-adds differently per shape.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_helpers import pre_collision_from_state, rel_err, say
from workload import droplet_rho

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1906_11027_amd import Sim  # noqa: E402
from paper_1906_11027_amd import sc_lbm as B  # noqa: E402

TOL = {"fp32": (1e-5, 1e-3), "fp64": (1e-11, 1e-9)}
# absolute velocity floor: the FP32 state resolves momentum to about its ulp
# times rho (2^-24 ~ 6e-8), which matters where max |u| itself is tiny
UFLOOR = {"fp32": 1e-7, "fp64": 1e-15}


def _compare(sim, orc, prec, label, floor=True):
    """floor=False: the velocity must meet the relative tolerance alone (the
    absolute FP32 floor is not needed where max |u| is well above it)."""
    got = sim.observe()
    ref = orc.fields()
    er = rel_err(got["rho"], ref["rho"])
    umax = max(np.max(np.abs(ref["u"])), 1e-12)
    du = float(np.max(np.abs(got["u"] - ref["u"])))
    eu = du / umax
    say("%s: rho rel err %.3e, u err / max|u| %.3e (max|u| %.3e)" % (label, er, eu, umax))
    tr, tu = TOL[prec]
    assert er <= tr, (label, er)
    assert du <= tu * umax + (UFLOOR[prec] * float(np.max(ref["rho"])) if floor else 0.0), (label, eu)
    return got, ref


# --------------------------------------------------------------- D2Q9 -----

@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("order", [4, 6, 8, 10])
def test_d2q9_droplet_64(order, prec):
    """The 64^2 droplet (R = 16, G = -5, tau = 1) pointwise up to 1,000
    steps, without the absolute velocity floor (max |u| ~ 5e-3 here)."""
    say("case d2q9 64x64 order", order, prec)
    rho0 = droplet_rho((64, 64), 16, seed=1)
    sim = Sim(rho0, "D2Q9", order=order, precision=prec)
    orc = O.Oracle(rho0, "D2Q9", order=order)
    for steps in (1, 49, 50, 100, 300, 500):
        sim.step(steps)
        orc.step(steps)
        _compare(sim, orc, prec, "E%d %s t=%d" % (order, prec, orc.steps), floor=False)
    sim.close()


@pytest.mark.parametrize("variant", list(range(9, 17)))
@pytest.mark.parametrize("shape,order", [((37, 29), 10), ((3, 5), 4), ((1, 16), 6), ((64, 64), 8)])
def test_d2q9_two_step_shapes(shape, order, variant):
    """Shapes that fuse two steps per launch, on ragged and tiny grids, with
    odd step counts (the last step runs single) and graph-replayed runs."""
    say("case two-step shape", variant, shape, order)
    rho0 = droplet_rho(shape, min(shape) / 3.0, seed=6)
    orc = O.Oracle(rho0, "D2Q9", order=order, tau=0.9)
    sim = Sim(rho0, "D2Q9", order=order, precision="fp64", tau=0.9, variant=variant)
    sim32 = Sim(rho0, "D2Q9", order=order, precision="fp32", tau=0.9, variant=variant)
    assert sim.variant.startswith("tile2")
    for steps in (1, 6, 33, 40):
        sim.step(steps)
        sim32.step(steps)
        orc.step(steps)
        _compare(sim, orc, "fp64", "%s %s E%d fp64 t=%d" % (sim.variant, shape, order, orc.steps))
        _compare(sim32, orc, "fp32", "%s %s E%d fp32 t=%d" % (sim.variant, shape, order, orc.steps))
    sim.close()
    sim32.close()


@pytest.mark.parametrize("shape,order", [((37, 29), 10), ((8, 8), 8), ((3, 5), 4), ((1, 16), 6),
                                         ((130, 67), 8)])
def test_d2q9_ragged_and_tiny(shape, order):
    say("case d2q9 ragged", shape, order)
    rho0 = droplet_rho(shape, min(shape) / 3.0, seed=5)
    for prec in ("fp32", "fp64"):
        sim = Sim(rho0, "D2Q9", order=order, precision=prec, tau=0.8)
        orc = O.Oracle(rho0, "D2Q9", order=order, tau=0.8)
        sim.step(40)
        orc.step(40)
        _compare(sim, orc, prec, "%s E%d %s" % (shape, order, prec))
        sim.close()


@pytest.mark.parametrize("order", [4, 10])
def test_d2q9_variants(order):
    """Every launch shape matches the oracle (FP64 state, ragged 100 x 77
    grid) and the FP32 shapes agree with each other to rounding."""
    say("case d2q9 variants", order)
    rho0 = droplet_rho((100, 77), 20, seed=9)
    orc = O.Oracle(rho0, "D2Q9", order=order).step(25)
    ref = None
    for v in range(B.sc_lbm_num_variants(B.make_params("D2Q9"))):
        sim = Sim(rho0, "D2Q9", order=order, variant=v, precision="fp64")
        sim.step(25)
        _compare(sim, orc, "fp64", "variant %s" % sim.variant)
        sim.close()
        sim = Sim(rho0, "D2Q9", order=order, variant=v)
        sim.step(25)
        st = sim.state()
        sim.close()
        if ref is None:
            ref = st
        else:
            d = float(np.max(np.abs(st - ref)))
            say("variant %d vs 0: max |diff| %.3e, bitwise %s" % (v, d, np.array_equal(st, ref)))
            assert d <= 1e-6


def test_d2q9_one_step_from_evolved_state():
    """Oracle restarted from the GPU's state at t = 300 reproduces the GPU's
    step t -> t + 1 (sampled one-step parity on developed fields)."""
    rho0 = droplet_rho((64, 48), 14, seed=2)
    sim = Sim(rho0, "D2Q9", order=8, precision="fp64")
    sim.step(300)
    orc = O.Oracle(rho0, "D2Q9", order=8)
    orc.set_f(pre_collision_from_state(sim, orc.c))
    sim.step(1)
    orc.step(1)
    _compare(sim, orc, "fp64", "restart E8")
    sim.close()


def test_force_on_analytic_psi():
    """sc_lbm_force on a given psi field equals Eq. (1) in the oracle."""
    x, y = np.meshgrid(np.arange(48.0), np.arange(40.0), indexing="ij")
    psi = 0.6 + 0.3 * np.sin(2 * np.pi * x / 48) * np.cos(4 * np.pi * y / 40)
    for order in (4, 6, 8, 10):
        for prec, tol in (("fp32", 2e-6), ("fp64", 1e-14)):
            sim = Sim(np.ones((48, 40)), "D2Q9", order=order, precision=prec)
            F = sim.force(psi)
            ref = O.force(psi, "D2Q9", order)
            err = np.max(np.abs(F - ref)) / np.max(np.abs(ref))
            say("force E%d %s err %.2e" % (order, prec, err))
            assert err < tol
            sim.close()


def test_init_state_and_observables():
    rho0 = droplet_rho((64, 64), 16, seed=1)
    sim = Sim(rho0, "D2Q9", order=4, precision="fp64")
    got = sim.observe()
    orc = O.Oracle(rho0, "D2Q9", order=4)
    ref = orc.fields()
    assert np.max(np.abs(got["rho"] - rho0)) < 1e-14
    assert np.max(np.abs(got["u"] - ref["u"])) < 1e-14
    ob, ro = got["obs"], orc.observables()
    for k in ("mass", "max_u", "mean_u", "l2_u", "rho_in", "rho_out", "p_in", "p_out", "dp", "radius", "rho_min",
              "rho_max"):
        assert abs(ob[k] - ro[k]) <= 1e-12 * max(1.0, abs(ro[k])), k
    sim.close()


def test_observables_parity_fp32():
    rho0 = droplet_rho((64, 64), 16, seed=1)
    sim = Sim(rho0, "D2Q9", order=4)
    orc = O.Oracle(rho0, "D2Q9", order=4)
    sim.step(500)
    orc.step(500)
    ob, ro = sim.observe(fields=False)["obs"], orc.observables()
    say("obs fp32:", {k: (ob[k], ro[k]) for k in ("max_u", "mean_u", "dp", "radius")})
    assert abs(ob["mass"] - ro["mass"]) < 1e-6 * ro["mass"]
    for k in ("max_u", "mean_u", "l2_u"):
        assert abs(ob[k] - ro[k]) < 1e-3 * ro[k], k
    assert abs(ob["dp"] - ro["dp"]) < 1e-4 * abs(ro["dp"]) + 1e-7
    for k in ("rho_min", "rho_max"):
        assert abs(ob[k] - ro[k]) < 1e-5 * ro[k], k
    sim.close()


@pytest.mark.parametrize("item", [
    dict(side=139, R=13, G=-5.171971471204614, tau=0.8, order=4, seed=1037),
    dict(side=154, R=19, G=-5.484176154757755, tau=1.2, order=6, seed=1018),
])
def test_fp32_run_stops_at_its_resolution(item):
    """Two droplets of the sweep whose FP32 runs never meet the 1e-10 rule:
    their max|u| keeps changing by ~1e-7 per check, the velocity the FP32
    state resolves (not round-off of max|u| itself).  The FP32 run stops on
    its resolution floor, at the steady state the FP64 run reaches with the
    literal rule: max|u|, the Laplace jump and the density extremes agree to
    the FP32 parity tolerances."""
    rho0 = droplet_rho((item["side"],) * 2, item["R"], seed=item["seed"])
    kw = dict(order=item["order"], G=item["G"], tau=item["tau"])
    a = Sim(rho0, "D2Q9", **kw)
    rc, n32 = a.step(150000, tol=1e-10)
    o32 = a.observe(fields=False)["obs"]
    a.close()
    b = Sim(rho0, "D2Q9", precision="fp64", **kw)
    rc64, n64 = b.step(250000, tol=1e-10)
    o64 = b.observe(fields=False)["obs"]
    b.close()
    say("fp32 stops after %d steps (by %d), fp64 after %d; max_u %.6e / %.6e, dp %.6e / %.6e" % (
        n32, o32["converged_by"], n64, o32["max_u"], o64["max_u"], o32["dp"], o64["dp"]))
    assert rc == 0 and rc64 == 0 and n32 < 150000 and n64 < 250000
    assert o32["converged_by"] == 2 and o64["converged_by"] == 1
    assert abs(o32["max_u"] - o64["max_u"]) < 1e-3 * o64["max_u"]
    assert abs(o32["dp"] - o64["dp"]) < 1e-4 * abs(o64["dp"]) + 1e-7
    for k in ("rho_min", "rho_max"):
        assert abs(o32[k] - o64[k]) < 1e-5 * o64[k], k


# -------------------------------------------------------------- D3Q19 -----

@pytest.mark.parametrize("collision", ["srt", "mrt"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_d3q19_droplet(order, collision):
    say("case d3q19", order, collision)
    rho0 = droplet_rho((20, 18, 13), 5, seed=3)
    for prec in ("fp32", "fp64"):
        sim = Sim(rho0, "D3Q19", order=order, collision=collision, precision=prec, tau=0.9)
        orc = O.Oracle(rho0, "D3Q19", order=order, collision=collision, tau=0.9)
        sim.step(30)
        orc.step(30)
        _compare(sim, orc, prec, "D3Q19 E%d %s %s" % (order, collision, prec))
        sim.close()


@pytest.mark.parametrize("order,collision,prec", [(8, "mrt", "fp32"), (4, "srt", "fp64"), (6, "mrt", "fp64")])
def test_d3q19_variants_agree(order, collision, prec):
    """Every launch shape (register window, prefetch, re-pull) against the
    oracle, and against shape 0 to rounding: the shapes do the same
    arithmetic on the same values, but the compiler may fuse multiply-adds
    differently per shape.  The z range (35) is not a multiple of the
    segment lengths, so the last segment of each shape overhangs the grid."""
    rho0 = droplet_rho((40, 21, 35), 8, seed=4)
    kw = dict(order=order, collision=collision, tau=0.9)
    orc = O.Oracle(rho0, "D3Q19", **kw).step(6)
    ref = None
    for v in range(B.sc_lbm_num_variants(B.make_params("D3Q19", (8, 8, 8)))):
        say("d3q19 variant", v, order, collision, prec)
        sim = Sim(rho0, "D3Q19", precision=prec, variant=v, **kw)
        sim.step(6)
        st = sim.state().astype(np.float64)
        _compare(sim, orc, prec, "D3Q19 E%d %s %s variant %s" % (order, collision, prec, sim.variant))
        sim.close()
        if ref is None:
            ref = st
        else:
            d = float(np.max(np.abs(st - ref)))
            say("  max |state - state of shape 0| = %.3e" % d)
            assert d <= (2e-6 if prec == "fp32" else 1e-14) * float(np.max(np.abs(ref))), (v, d)


def test_d3q19_persistent_march_generations():
    """The persistent march takes column segments in generations of the
    blocks that fit at once (one 512-thread block per CU).  A 192 x 64 x 192
    grid has 3 x 8 x 12 = 288 segments of 64 x 8 x 16 nodes, more than one
    generation; the persistent shape must give the state of the
    one-segment-per-block shape, which does the same arithmetic per node."""
    from paper_1906_11027_amd import sc_lbm as B
    rho0 = droplet_rho((192, 64, 192), 20, seed=6)
    states = {}
    for v in ("march64x8r1h16pf1", "pmarch64x8r1h16pf1"):
        idx = next(i for i in range(B.sc_lbm_num_variants(B.make_params("D3Q19", (8, 8, 8))))
                   if _d3q19_variant_name(i) == v)
        sim = Sim(rho0, "D3Q19", order=8, collision="mrt", variant=idx)
        assert sim.variant == v
        sim.step(12)
        states[v] = sim.state().astype(np.float64)
        sim.close()
    a, b = states["march64x8r1h16pf1"], states["pmarch64x8r1h16pf1"]
    d = float(np.max(np.abs(a - b)))
    say("persistent vs one-segment-per-block march, 288 segments: max |diff| %.2e" % d)
    assert d <= 2e-6 * float(np.max(np.abs(a)))


def _d3q19_variant_name(i):
    """Name of D3Q19 launch shape i (from a throwaway 8^3 handle)."""
    sim = Sim(droplet_rho((8, 8, 8), 2, seed=1), "D3Q19", order=4, variant=i)
    name = sim.variant
    sim.close()
    return name


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("order", [4, 8])
def test_d3q19_mrt_distinct_rates(order, prec):
    """Bulk and ghost rates that differ from each other and from 1/tau
    (0.7, 1.6, tau = 0.9), so every moment correction of the MRT collision,
    the bulk one included, changes the result."""
    say("case d3q19 mrt s_bulk 0.7 s_ghost 1.6", order, prec)
    rho0 = droplet_rho((20, 18, 13), 5, seed=5)
    kw = dict(order=order, collision="mrt", tau=0.9, s_bulk=0.7, s_ghost=1.6)
    sim = Sim(rho0, "D3Q19", precision=prec, **kw)
    orc = O.Oracle(rho0, "D3Q19", **kw)
    sim.step(30)
    orc.step(30)
    _compare(sim, orc, prec, "D3Q19 E%d mrt 0.7/1.6 %s" % (order, prec))
    sim.close()


def test_d3q19_mrt_equals_srt_when_rates_equal():
    rho0 = droplet_rho((16, 16, 16), 5, seed=3)
    a = Sim(rho0, "D3Q19", order=8, collision="srt", precision="fp64", tau=0.8)
    b = Sim(rho0, "D3Q19", order=8, collision="mrt", precision="fp64", tau=0.8,
            s_bulk=1.25, s_ghost=1.25)
    a.step(20)
    b.step(20)
    assert np.max(np.abs(a.state() - b.state())) < 1e-13
    a.close()
    b.close()


# -------------------------------------------------- runtime behaviour -----

def test_graph_and_direct_launch_agree():
    rho0 = droplet_rho((64, 64), 16, seed=1)
    a = Sim(rho0, "D2Q9", order=8)
    b = Sim(rho0, "D2Q9", order=8)
    a.step(96)          # graph-captured chunks of 32
    for _ in range(96):
        b.step(1)       # direct launches
    assert np.array_equal(a.state(), b.state())
    a.close()
    b.close()


def test_checkpoint_resume_bitwise():
    rho0 = droplet_rho((64, 64), 16, seed=1)
    a = Sim(rho0, "D2Q9", order=6)
    a.step(70)
    f = a.state()
    a.step(45)
    b = Sim(rho0, "D2Q9", order=6)
    b.set_state(f, 70)
    b.step(45)
    assert np.array_equal(a.state(), b.state())
    assert b.observe(fields=False)["obs"]["step"] == 115
    a.close()
    b.close()


def test_convergence_loop_and_nonfinite():
    rho0 = droplet_rho((32, 32), 8, seed=1)
    sim = Sim(rho0, "D2Q9", order=4, obs_every=50)
    rc, done = sim.step(20000, tol=1e-7)
    assert rc == B.SC_OK
    assert 0 < done < 20000
    f = sim.state()
    f[5] = np.nan
    sim.set_state(f, 0)
    rc, done = sim.step(200, tol=1e-9)
    assert rc == B.SC_E_NONFINITE
    sim.close()


def test_mass_conservation_fp32():
    rho0 = droplet_rho((64, 64), 16, seed=1)
    sim = Sim(rho0, "D2Q9", order=8)
    m0 = sim.observe(fields=False)["obs"]["mass"]
    sim.step(10000)
    ob = sim.observe(fields=False)["obs"]
    say("fp32 mass drift over 1e4 steps: %.2e rel" % ((ob["mass"] - m0) / m0))
    assert abs(ob["mass"] - m0) < 1e-5 * m0
    sim.close()


def test_mass_conservation_fp64():
    rho0 = droplet_rho((64, 64), 16, seed=1)
    sim = Sim(rho0, "D2Q9", order=8, precision="fp64")
    m0 = sim.observe(fields=False)["obs"]["mass"]
    sim.step(5000)
    ob = sim.observe(fields=False)["obs"]
    assert abs(ob["mass"] - m0) < 1e-12 * m0
    sim.close()


@pytest.mark.parametrize("order", [4, 8])
def test_droplet_64_long_horizon_observables(order):
    """64^2 droplet (R = 16, G = -5, tau = 1) for 10,000 steps: FP32 GPU
    spurious-velocity norms and Laplace jump against the FP64 oracle; the
    FP64 GPU state pointwise."""
    rho0 = droplet_rho((64, 64), 16, seed=1)
    orc = O.Oracle(rho0, "D2Q9", order=order).step(10000)
    ro = orc.observables()
    ref = orc.fields()
    s32 = Sim(rho0, "D2Q9", order=order)
    s32.step(10000)
    ob = s32.observe(fields=False)["obs"]
    say("E%d 1e4 steps fp32 vs oracle: max_u %.6e/%.6e mean_u %.6e/%.6e dp %.6e/%.6e" % (
        order, ob["max_u"], ro["max_u"], ob["mean_u"], ro["mean_u"], ob["dp"], ro["dp"]))
    for k in ("max_u", "mean_u", "l2_u"):
        assert abs(ob[k] - ro[k]) <= 1e-3 * ro[k], k
    assert abs(ob["dp"] - ro["dp"]) <= 1e-4 * abs(ro["dp"])
    assert abs(ob["radius"] - ro["radius"]) <= 1e-4 * ro["radius"]
    s32.close()
    s64 = Sim(rho0, "D2Q9", order=order, precision="fp64")
    s64.step(10000)
    got = s64.observe()
    er = rel_err(got["rho"], ref["rho"])
    say("E%d 1e4 steps fp64 pointwise rho err %.2e" % (order, er))
    assert er <= 1e-11
    s64.close()


# ------------------------------------------------------------ batches -----

def _batch_items():
    from workload import sweep_items
    its = sweep_items(6, seed=11, side_range=(20, 70))
    out = []
    for k, it in enumerate(its):
        side = it["side"]
        shape = (side, side - 3 * k)          # ragged, non-square grids
        out.append({"rho0": droplet_rho(shape, min(it["R"], min(shape) // 3), seed=it["seed"]),
                    "order": it["order"], "G": it["G"], "tau": it["tau"]})
    return out


@pytest.mark.parametrize("shape", [-1, 0, 1, 2, 3])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_matches_oracle_and_single(prec, shape):
    """Every batched launch shape (one step per launch; two per launch on
    32 x 8, 64 x 16 and 32 x 16 tiles; -1 automatic) against the oracle and
    the single-grid runs.  61 steps: the two-step shapes end on a one-step
    launch."""
    from paper_1906_11027_amd import Batch
    items = _batch_items()
    say("batch shape %d %s items:" % (shape, prec),
        [(it["rho0"].shape, it["order"], round(it["G"], 3), it["tau"]) for it in items])
    bt = Batch(items, precision=prec, variant=shape)
    bt.step(61)
    for k, it in enumerate(items):
        orc = O.Oracle(it["rho0"], "D2Q9", order=it["order"], G=it["G"], tau=it["tau"]).step(61)
        got, ref = bt.observe(k), orc.fields()
        er = rel_err(got["rho"], ref["rho"])
        eu = float(np.max(np.abs(got["u"] - ref["u"])) / max(np.max(np.abs(ref["u"])), 1e-12))
        say("batch item %d %s: rho %.2e u %.2e" % (k, it["rho0"].shape, er, eu))
        tr, tu = TOL[prec]
        assert er <= tr and eu <= tu, (k, er, eu)
        single = Sim(it["rho0"], "D2Q9", order=it["order"], G=it["G"], tau=it["tau"], precision=prec,
                     rho_ref=bt.rho_ref)
        single.step(61)
        sg = single.observe()
        assert np.max(np.abs(sg["rho"] - got["rho"])) <= (1e-6 if prec == "fp32" else 1e-13)
        single.close()
    bt.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_autotune(prec):
    """The batched shape tuner returns one of the batched shapes with a
    positive time per step, and a batch built with its choice matches the
    automatic shape's result to rounding."""
    from paper_1906_11027_amd import Batch, batch_autotune
    from paper_1906_11027_amd import sc_lbm as B
    items = _batch_items()
    v, ms = batch_autotune(items, steps=32, precision=prec)
    say("batch autotune %s: variant %d, %.4f ms per step" % (prec, v, ms))
    assert 0 <= v < B.lib().sc_lbm_batch_num_variants() and ms > 0
    a = Batch(items, precision=prec, variant=v)
    b = Batch(items, precision=prec)
    say("  tuned %s, automatic %s" % (a.variant, b.variant))
    a.step(40)
    b.step(40)
    for k in range(len(items)):
        ra, rb = a.observe(k)["rho"], b.observe(k)["rho"]
        assert np.max(np.abs(ra - rb)) <= (1e-6 if prec == "fp32" else 1e-13) * np.max(np.abs(rb)), k
    a.close()
    b.close()


def test_batch_convergence_and_quarantine():
    from paper_1906_11027_amd import Batch
    items = [{"rho0": droplet_rho((40, 40), 10, seed=1), "order": 4},
             {"rho0": droplet_rho((48, 36), 9, seed=2), "order": 8, "tau": 0.8},
             # far past the stable range: diverges and must be quarantined
             {"rho0": droplet_rho((32, 32), 8, seed=3), "order": 4, "G": -30.0, "tau": 0.51}]
    # the batched two-step shape on 32 x 8 tiles runs the arithmetic of the
    # single-grid shape tile2x32x8 (variant 10), so a retired item can be
    # checked against a single run to FP32 rounding after ~10^4 steps
    bt = Batch(items, obs_every=50, variant=1)
    rc, done = bt.step(200000, tol=1e-7)
    st = [bt.status(k) for k in range(3)]
    say("batch status:", st, "steps", done)
    assert bt.active == 0
    assert st[0][1] in (1, 2) and st[1][1] in (1, 2)
    assert st[2][1] == -1
    # retired items keep their state: a converged item matches a single run
    # with the batch's storage shift
    single = Sim(items[0]["rho0"], "D2Q9", order=4, rho_ref=bt.rho_ref, variant=10)
    single.step(st[0][0])
    a = single.observe()["rho"]
    b = bt.observe(0)["rho"]
    assert np.max(np.abs(a - b)) < 1e-6
    single.close()
    bt.close()


def test_autotune_picks_a_variant_and_is_used():
    p = B.make_params("D2Q9", (96, 80), order=6)
    v, ms = B.sc_lbm_autotune(p, steps=10)
    assert 0 <= v < B.sc_lbm_num_variants(p) and ms > 0
    sim = Sim(droplet_rho((96, 80), 20, seed=1), "D2Q9", order=6)
    names = []
    for k in range(B.sc_lbm_num_variants(p)):
        s2 = Sim(np.ones((96, 80)), "D2Q9", order=6, variant=k)
        names.append(s2.variant)
        s2.close()
    assert sim.variant == names[v]
    sim.close()
