"""Pins for the oracle's solid walls: standard (full-way) bounce-back with a
virtual wall density in the interaction force (Sec. 3, droplet on a wall)."""
import warnings
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import eos as E
from oracle import oracle as O
from tests.exact_step import exact_steps

warnings.simplefilter("ignore")


def _walls(shape, layers):
    """Bottom and top walls `layers` nodes thick (y axis)."""
    m = np.zeros(shape, dtype=bool)
    m[:, :layers] = True
    m[:, shape[1] - layers:] = True
    return m


@pytest.mark.parametrize("lattice,order,forcing", [("D2Q9", 4, "guo"), ("D2Q9", 8, "edm"),
                                                   ("D2Q25", 8, "guo"), ("D2Q13", 6, "edm")])
def test_exact_steps_with_walls(lattice, order, forcing):
    """Three steps against the exact-rational statement (push streaming,
    dict nodes) with two-layer walls, psi = rho and rho_w = 3/2 (G = -2
    keeps every fluid density in 0.5 .. 2, where 1/rho does not amplify the
    FP64 rounding)."""
    shape = (6, 9)
    rng = np.random.default_rng(7)
    vals = rng.integers(20, 120, size=shape)
    solid = _walls(shape, 2)
    rho_ex = {idx: Fr(int(v), 64) for idx, v in np.ndenumerate(vals)}
    sset = {idx for idx, v in np.ndenumerate(solid) if v}
    fex = exact_steps(rho_ex, shape, lattice, order, -2, Fr(1, 3), Fr(9, 10), 3, forcing=forcing,
                      solid=sset, rho_w=Fr(3, 2))
    o = O.Oracle(vals / 64.0, lattice, order=order, G=-2.0, psi="identity", tau=0.9, forcing=forcing)
    o.set_walls(solid, 1.5)
    o.step(3)
    f = o.get_f()
    ex = np.zeros_like(f)
    for idx in np.ndindex(*shape):
        for q, v in enumerate(fex[idx]):
            ex[(q,) + idx] = float(v)
    assert np.max(np.abs(f - ex)) < 1e-14 * np.max(np.abs(ex))


def test_fluid_at_rest_between_walls_stays_at_rest():
    """Uniform fluid at rest with no interaction, walls holding the same
    equilibrium: f = feq(rho, 0) with bounce-back is an exact steady state
    (no spurious wall flow), also with the interaction on when psi_w is
    the fluid's own psi (a wall indistinguishable from the fluid)."""
    shape = (12, 10)
    for G, rw in ((0.0, 0.7), (-4.0, 1.3)):
        o = O.Oracle(np.full(shape, 1.3), "D2Q25", order=8, G=G, tau=0.8)
        o.set_walls(_walls(shape, 2), rw)
        o.step(200)
        fl = o.fields()
        assert np.abs(fl["u"]).max() < 1e-15
        assert np.abs(fl["rho"] - 1.3).max() < 1e-14


def test_total_mass_conserved_with_walls():
    shape = (40, 30)
    solid = _walls(shape, 2)
    rho0 = np.full(shape, 0.5)
    x, y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    rho0[(x - 20) ** 2 + (y - 2) ** 2 < 100] = 2.0
    o = O.Oracle(rho0, "D2Q9", order=8, G=-5.0, tau=1.0)
    o.set_walls(solid, 1.0)
    m0 = o.get_f().sum()
    o.step(1500)
    f = o.get_f()
    assert abs(f.sum() - m0) < 1e-12 * m0
    assert np.all(np.isfinite(f))


def test_mirror_symmetry_of_a_wall_droplet():
    """A droplet sitting on the bottom wall, symmetric about x = xc, stays
    symmetric (no jitter): rho(xc + d) = rho(xc - d)."""
    shape = (48, 32)
    solid = _walls(shape, 2)
    x, y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    r = np.sqrt((x - 24.0) ** 2 + (y - 2.0) ** 2)
    rho0 = 1.04 - 0.89 * np.tanh(2.0 * (r - 10.0) / 3.0)
    o = O.Oracle(rho0, "D2Q25", order=8, G=-5.0 * 12 / 7, tau=1.0, forcing="edm")
    o.set_walls(solid, 1.2)
    o.step(800)
    rho = o.fields()["rho"]
    mirror = rho[(48 - np.arange(48)) % 48, :]
    assert np.max(np.abs(rho - mirror)) < 1e-11 * rho.max()


def test_wettability_follows_wall_density():
    """Sec. 3: the virtual wall density tunes wettability.  A P-R droplet
    at T = 0.9 Tc (D2Q9, E4, EDM) spreads more on the denser wall: its base
    is wider and its apex lower for rho_w = 4.5 than for rho_w = 1.5."""
    eos = E.eos_params(0.9)
    rv, rl = E.maxwell(eos)
    shape = (80, 48)
    solid = _walls(shape, 2)
    x, y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    r = np.sqrt((x - 40.0) ** 2 + (y - 2.0) ** 2)
    rho0 = 0.5 * (rl + rv) - 0.5 * (rl - rv) * np.tanh(2.0 * (r - 15.0) / 4.0)
    shapes = {}
    for rw in (1.5, 4.5):
        o = O.Oracle(rho0, "D2Q9", order=4, G=-1.0, psi="pr", eos=eos, forcing="edm", tau=1.0)
        o.set_walls(solid, rw)
        o.step(6000)
        rho = o.fields()["rho"]
        mid = 0.5 * (rl + rv)
        base = int((rho[:, 2] > mid).sum())          # first fluid row
        height = int((rho[40, 2:-2] > mid).sum())    # centre column
        shapes[rw] = (base, height)
    assert shapes[4.5][0] > shapes[1.5][0] and shapes[4.5][1] < shapes[1.5][1], shapes
