"""GPU parity of the any-lattice 2D family against the FP64 oracle: the
D2Q13 / D2Q25 lattices of Sec. 3 (Table 1), the exact difference method
forcing and the Peng-Robinson pseudo-potential of the paper's experiments.

Tolerances as for D2Q9 (tests/test_gpu_parity.py): FP64 state <= 1e-11
pointwise; FP32 state density <= 1e-5 relative and velocity <= 1e-3 of
max |u| (plus the FP32 momentum resolution, 1e-7 max rho, where max |u| is
itself near round-off) at horizons up to 100 steps.
"""
import warnings

import numpy as np
import pytest

from oracle import eos as E
from oracle import oracle as O
from tests.gpu_helpers import pre_collision_from_state, rel_err, say
from workload import droplet_rho, slab_rho

pytestmark = pytest.mark.gpu
warnings.simplefilter("ignore")

torch = pytest.importorskip("torch")

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1906_11027_amd import Sim  # noqa: E402
from paper_1906_11027_amd import sc_lbm as B  # noqa: E402

TOL = {"fp32": (1e-5, 1e-3), "fp64": (1e-11, 1e-9)}
CS2 = {"D2Q9": 1 / 3, "D2Q13": 2 / 5, "D2Q25": 4 / 7}


def g_scaled(lattice):
    """G = -15 cs2: the exp-psi EOS p / cs2 is then the same function of rho
    on every lattice (the D2Q9 value G = -5), so the droplet separates."""
    return -15.0 * CS2[lattice]


# absolute velocity floor: the FP32 state resolves momentum to about its
# ulp times rho (2^-24 ~ 6e-8), which matters where max |u| itself is tiny
UFLOOR = {"fp32": 1e-7, "fp64": 1e-15}


def _compare(sim, orc, prec, label):
    got = sim.observe()
    ref = orc.fields()
    er = rel_err(got["rho"], ref["rho"])
    umax = max(np.max(np.abs(ref["u"])), 1e-12)
    du = float(np.max(np.abs(got["u"] - ref["u"])))
    say("%s: rho rel err %.3e, u err / max|u| %.3e (max|u| %.3e)" % (label, er, du / umax, umax))
    tr, tu = TOL[prec]
    assert er <= tr, (label, er)
    assert du <= tu * umax + UFLOOR[prec] * float(np.max(ref["rho"])), (label, du / umax)
    return got, ref


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("forcing", ["guo", "edm"])
@pytest.mark.parametrize("lattice,order", [("D2Q13", 6), ("D2Q25", 8), ("D2Q13", 10), ("D2Q25", 4)])
def test_wide_droplet(lattice, order, forcing, prec):
    """Ragged 70 x 53 droplet, exp psi with G scaled to the lattice's cs2."""
    say("case wide droplet", lattice, order, forcing, prec)
    rho0 = droplet_rho((70, 53), 14, seed=11)
    kw = dict(order=order, G=g_scaled(lattice), tau=0.9, forcing=forcing)
    sim = Sim(rho0, lattice, precision=prec, **kw)
    orc = O.Oracle(rho0, lattice, **kw)
    for steps in (1, 29, 70):
        sim.step(steps)
        orc.step(steps)
        _compare(sim, orc, prec, "%s E%d %s %s t=%d" % (lattice, order, forcing, prec, orc.steps))
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("order", [4, 8])
def test_d2q9_edm(order, prec):
    say("case d2q9 edm", order, prec)
    rho0 = droplet_rho((64, 48), 12, seed=12)
    sim = Sim(rho0, "D2Q9", order=order, precision=prec, forcing="edm", tau=0.8)
    orc = O.Oracle(rho0, "D2Q9", order=order, forcing="edm", tau=0.8)
    sim.step(100)
    orc.step(100)
    _compare(sim, orc, prec, "D2Q9 E%d edm %s" % (order, prec))
    sim.close()


@pytest.mark.parametrize("lattice", ["D2Q9", "D2Q13", "D2Q25"])
def test_wide_variants_and_state_layout(lattice):
    """Every launch shape matches the oracle (FP64 state), its FP32 states
    agree to rounding (the shapes' instruction schedules contract different
    multiply-adds, so they need not agree bitwise), and the FP64 state mapped
    to pre-collision distributions is the oracle's."""
    rho0 = droplet_rho((91, 45), 12, seed=13)
    kw = dict(order=8, G=g_scaled(lattice), tau=0.85, forcing="edm")
    orc = O.Oracle(rho0, lattice, **kw)
    orc.step(21)
    ref = None
    nv = B.sc_lbm_num_variants(B.make_params(lattice, forcing="edm"))
    for v in range(nv):
        sim = Sim(rho0, lattice, variant=v, precision="fp64", **kw)
        sim.step(21)
        _compare(sim, orc, "fp64", "%s variant %s" % (lattice, sim.variant))
        sim.close()
        sim = Sim(rho0, lattice, variant=v, **kw)
        sim.step(21)
        st = sim.state()
        sim.close()
        if ref is None:
            ref = st
        else:
            d = float(np.max(np.abs(st - ref)))
            say("variant %d vs 0: max |diff| %.3e, bitwise %s" % (v, d, np.array_equal(st, ref)))
            assert d <= 1e-6
    sim = Sim(rho0, lattice, precision="fp64", **kw)
    sim.step(21)
    oc = O.lattice_table(lattice)[1]
    f_gpu = pre_collision_from_state(sim, oc)
    f_orc = orc.get_f()
    err = float(np.max(np.abs(f_gpu - f_orc)))
    say("%s state vs oracle f: %.3e" % (lattice, err))
    assert err < 1e-12
    sim.close()


@pytest.mark.parametrize("lattice,forcing", [("D2Q9", "guo"), ("D2Q13", "edm"), ("D2Q25", "edm")])
def test_two_step_interior_and_edge_tiles(lattice, forcing):
    """Every launch shape on a ragged 283 x 61 grid, large enough that each
    two-step shape (tiles up to 128 x 8 and 64 x 16) has tiles whose pulled
    region lies inside the grid (unwrapped addresses) beside tiles at its
    edge (wrapped ones): FP64 state against the oracle after 13 steps (six
    two-step launches and a one-step one)."""
    rho0 = droplet_rho((283, 61), 20, seed=14)
    kw = dict(order=8, G=g_scaled(lattice), tau=0.85, forcing=forcing)
    orc = O.Oracle(rho0, lattice, **kw)
    orc.step(13)
    for v in range(B.sc_lbm_num_variants(B.make_params(lattice, forcing=forcing))):
        say("case interior/edge tiles", lattice, forcing, "variant", v)
        sim = Sim(rho0, lattice, variant=v, precision="fp64", **kw)
        sim.step(13)
        _compare(sim, orc, "fp64", "%s %s variant %s" % (lattice, forcing, sim.variant))
        sim.close()


@pytest.mark.parametrize("variant", [-1, 6, 9])
@pytest.mark.parametrize("shape", [(3, 5), (1, 9), (2, 2), (33, 7)])
@pytest.mark.parametrize("lattice", ["D2Q13", "D2Q25"])
def test_wide_tiny_grids(lattice, shape, variant):
    """Grids narrower than the streaming reach (2) and the force stencil wrap
    several times around the periodic box; also in the two-step shapes,
    whose halos (2R + M = 8 nodes) wrap several times (31 steps: the last
    launch is a one-step one)."""
    say("case wide tiny", lattice, shape, variant)
    rng = np.random.default_rng(sum(shape))
    rho0 = 1.0 + 0.3 * rng.random(shape)
    kw = dict(order=10, G=-2.0, tau=0.9)
    for prec in ("fp32", "fp64"):
        sim = Sim(rho0, lattice, precision=prec, variant=variant, **kw)
        orc = O.Oracle(rho0, lattice, **kw)
        sim.step(31)
        orc.step(31)
        _compare(sim, orc, prec, "%s %s %s" % (lattice, shape, prec))
        sim.close()


def _pr(Tr=0.85):
    eos = E.eos_params(Tr)
    return {k: eos[k] for k in ("a", "b", "R", "T", "alpha")}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("lattice,order", [("D2Q9", 4), ("D2Q9", 8), ("D2Q25", 8), ("D2Q13", 6)])
def test_pr_droplet_edm(lattice, order, prec):
    """The droplet of Sec. 3 (60 x 60, r0 = 15, P-R psi, EDM) at T/Tc = 0.85."""
    say("case pr droplet", lattice, order, prec)
    eos = _pr(0.85)
    rv, rl = E.maxwell(E.eos_params(0.85))
    rho0 = droplet_rho((60, 60), 15, rho_l=rl, rho_v=rv, seed=14)
    kw = dict(order=order, G=-1.0, psi="pr", eos=eos, forcing="edm", tau=1.0)
    sim = Sim(rho0, lattice, precision=prec, **kw)
    orc = O.Oracle(rho0, lattice, **kw)
    for steps in (1, 99):
        sim.step(steps)
        orc.step(steps)
        _compare(sim, orc, prec, "P-R %s E%d %s t=%d" % (lattice, order, prec, orc.steps))
    ob, oo = sim.observe()["obs"], orc.observables()
    say("mass", ob["mass"], oo["mass"])
    assert abs(ob["mass"] - oo["mass"]) <= (1e-6 if prec == "fp32" else 1e-11) * oo["mass"]
    # p = cs2 rho + G c0 psi^2 / 2 is a small difference of two O(cs2 rho)
    # terms in the liquid: compare on the scale of cs2 rho_in
    scale = CS2[lattice] * oo["rho_in"]
    for k in ("p_in", "p_out"):
        say(k, ob[k], oo[k])
        assert abs(ob[k] - oo[k]) <= (2e-5 if prec == "fp32" else 1e-11) * scale
    sim.close()


def test_pr_slab_guo_fp64_long():
    """Flat P-R interface with Guo forcing, FP64 state, 2000 steps: pointwise
    parity over a long horizon with the Peng-Robinson psi."""
    eos = _pr(0.85)
    rv, rl = E.maxwell(E.eos_params(0.85))
    rho0 = slab_rho((80, 4), 40, rho_l=rl, rho_v=rv, width=4)
    kw = dict(order=4, G=-1.0, psi="pr", eos=eos, forcing="guo", tau=1.0)
    sim = Sim(rho0, "D2Q9", precision="fp64", **kw)
    orc = O.Oracle(rho0, "D2Q9", **kw)
    sim.step(2000)
    orc.step(2000)
    _compare(sim, orc, "fp64", "P-R slab guo 2000")
    sim.close()


@pytest.mark.parametrize("lattice", ["D2Q13", "D2Q25"])
def test_wide_force_entry_point(lattice):
    """sc_lbm_force with an analytic psi field on the wide lattices."""
    shape = (48, 40)
    x, y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    psi = 1.0 + 0.3 * np.cos(2 * np.pi * x / shape[0]) * np.sin(4 * np.pi * y / shape[1])
    sim = Sim(np.ones(shape), lattice, order=8, precision="fp64", G=-4.0, c0=0.4)
    F = sim.force(psi)
    ref = O.force(psi, lattice, order=8, G=-4.0, c0=0.4)
    assert np.max(np.abs(F - ref)) < 1e-13 * np.max(np.abs(ref))
    sim.close()


def test_wide_mass_conservation_fp32():
    """FP32 state over 3000 steps: mass is kept to the FP64 reduction's
    resolution of the FP32 state (the rest population closes the balance)."""
    rho0 = droplet_rho((96, 96), 24, seed=15)
    sim = Sim(rho0, "D2Q25", order=8, G=g_scaled("D2Q25"), tau=19 / 24, forcing="edm")
    m0 = sim.observe()["obs"]["mass"]
    sim.step(3000)
    ob = sim.observe()["obs"]
    say("D2Q25 fp32 mass drift", (ob["mass"] - m0) / m0, "max|u|", ob["max_u"])
    assert abs(ob["mass"] - m0) < 2e-6 * m0
    assert np.isfinite(ob["max_u"])
    sim.close()


def test_wide_rejections():
    """Unsupported combinations fail at create with SC_E_UNSUPPORTED."""
    rho0 = np.ones((8, 8, 8))
    with pytest.raises(B.ScError) as ei:
        Sim(rho0, "D3Q19", order=4, forcing="edm")
    assert ei.value.code == B.SC_E_UNSUPPORTED
    with pytest.raises(B.ScError) as ei:
        Sim(np.ones((8, 8)), "D2Q25", order=4, collision="mrt")
    assert ei.value.code == B.SC_E_UNSUPPORTED
    with pytest.raises(B.ScError) as ei:
        Sim(np.ones((8, 8)), "D2Q13", order=4, psi="pr", eos={"a": 0.04, "b": -1.0, "R": 1.0, "T": 0.06,
                                                             "alpha": 1.0})
    assert ei.value.code == B.SC_E_INVAL
