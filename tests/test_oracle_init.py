"""Pins for the oracle's two initial states: f = feq(rho0, 0) and the start
at rest in the forced sense, f = feq(rho0, -F / (2 rho0)), under which the
velocity the forcing schemes report, (sum f c + F/2) / rho (Guo, Eq. (4);
the exact difference method alike), is zero at t = 0."""
import warnings
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import eos as E
from oracle import oracle as O
from tests.exact_step import exact_steps
from workload import droplet_rho

warnings.simplefilter("ignore")

CASES = [
    ("D2Q9", (40, 34), dict(order=8, G=-5.0, tau=1.0)),
    ("D2Q13", (36, 30), dict(order=6, G=-5.0 * 6 / 5, tau=0.9, forcing="edm")),
    ("D2Q25", (36, 30), dict(order=8, G=-5.0 * 12 / 7, tau=0.8)),
    ("D3Q19", (14, 12, 10), dict(order=4, G=-5.0, tau=1.0, collision="mrt")),
]


def _psi_exp(rho):
    return 1.0 - np.exp(-rho)


@pytest.mark.parametrize("lattice,shape,kw", CASES)
def test_rest_start_has_zero_forced_velocity(lattice, shape, kw):
    rho0 = droplet_rho(shape, min(shape) / 4, seed=3)
    o = O.Oracle(rho0, lattice, init="rest", **kw)
    fl = o.fields()
    assert np.max(np.abs(fl["rho"] - rho0)) < 1e-14
    assert np.max(np.abs(fl["u"])) < 1e-15
    # the equilibrium start reports u = F / (2 rho) instead
    e = O.Oracle(rho0, lattice, **kw).fields()
    assert np.max(np.abs(e["u"] - e["F"] / (2 * rho0[None]))) < 1e-15
    assert np.max(np.abs(e["u"])) > 1e-3


@pytest.mark.parametrize("lattice,shape,kw", CASES)
def test_rest_start_moments(lattice, shape, kw):
    """Zeroth, first and second moments of the start against the force of
    Eq. (1) computed by the stand-alone force routine: rho0, -F/2 and
    rho0 cs2 I + rho0 v v with v = -F / (2 rho0)."""
    rho0 = droplet_rho(shape, min(shape) / 4, seed=4)
    o = O.Oracle(rho0, lattice, init="rest", **kw)
    f = o.get_f()
    dim, c, w, cs2 = O.lattice_table(lattice)
    F = O.force(_psi_exp(rho0), lattice, order=kw["order"], G=kw["G"])
    v = -F / (2 * rho0[None])
    assert np.max(np.abs(f.sum(axis=0) - rho0)) < 1e-14
    for a in range(dim):
        ja = np.tensordot(c[:, a].astype(float), f, axes=(0, 0))
        assert np.max(np.abs(ja + F[a] / 2)) < 1e-15
        for b in range(dim):
            pab = np.tensordot((c[:, a] * c[:, b]).astype(float), f, axes=(0, 0))
            ref = rho0 * (cs2 * (a == b) + v[a] * v[b])
            assert np.max(np.abs(pab - ref)) < 1e-14


def test_uniform_density_starts_agree():
    """No force on a uniform field: both starts are the same state."""
    rho0 = np.full((16, 12), 0.7)
    a = O.Oracle(rho0, "D2Q25", order=8, init="rest").get_f()
    b = O.Oracle(rho0, "D2Q25", order=8).get_f()
    assert np.array_equal(a, b)


def test_rest_start_with_peng_robinson_psi():
    e = E.eos_params(0.8)
    eos = {k: e[k] for k in ("a", "b", "R", "T", "alpha")}
    rv, rl = E.maxwell(e)
    rho0 = droplet_rho((40, 40), 10, rho_l=rl, rho_v=rv, width=4.0)
    o = O.Oracle(rho0, "D2Q13", order=6, G=-1.0, psi="pr", eos=eos, forcing="edm", tau=11 / 12, init="rest")
    assert np.max(np.abs(o.fields()["u"])) < 1e-15


@pytest.mark.parametrize("lattice,order,forcing,collision", [("D2Q9", 8, "guo", "srt"), ("D2Q13", 6, "edm", "srt"),
                                                             ("D3Q19", 4, "guo", "mrt")])
def test_rest_start_steps_match_exact_rational(lattice, order, forcing, collision):
    """Two steps from the rest start against the exact-rational statement
    (psi = rho, rational densities)."""
    shape = (5, 6) if lattice != "D3Q19" else (4, 3, 3)
    rng = np.random.default_rng(11)
    vals = rng.integers(40, 100, size=shape)
    rho_ex = {idx: Fr(int(v), 64) for idx, v in np.ndenumerate(vals)}
    kw = dict(s_bulk=Fr(6, 5), s_ghost=Fr(6, 5)) if collision == "mrt" else {}
    fex = exact_steps(rho_ex, shape, lattice, order, -2, Fr(1, 3), Fr(9, 10), 2, collision=collision,
                      forcing=forcing, init="rest", **kw)
    o = O.Oracle(vals / 64.0, lattice, order=order, G=-2.0, psi="identity", tau=0.9, forcing=forcing,
                 collision=collision, s_bulk=1.2, s_ghost=1.2, init="rest")
    o.step(2)
    f = o.get_f()
    ex = np.zeros_like(f)
    for idx in np.ndindex(*shape):
        for q, val in enumerate(fex[idx]):
            ex[(q,) + idx] = float(val)
    assert np.max(np.abs(f - ex)) < 1e-14 * np.max(np.abs(ex))


def test_rest_start_shortens_the_way_to_a_known_steady_state():
    """From the steady density of a 48^2 droplet, the rest start is already
    nearly steady; the equilibrium start first sends out the velocity
    impulse F / (2 rho) and takes longer to settle."""
    kw = dict(order=8, G=-5.0, tau=1.0)
    o = O.Oracle(droplet_rho((48, 48), 12), "D2Q9", **kw)
    o.step(6000)
    rs = o.fields()["rho"]
    us = o.fields()["u"]

    def dev(init):
        s = O.Oracle(rs, "D2Q9", init=init, **kw)
        s.step(200)
        return np.max(np.abs(s.fields()["u"] - us))
    assert dev("rest") < 0.5 * dev("equilibrium")
