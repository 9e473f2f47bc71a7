"""Pins for the oracle's time step (Sec. 2, Eq. (3)-(4); Sec. 4, Eq. (7)).

* exact-rational brute force on tiny grids, every stencil order, SRT and MRT;
* textbook moment identities of the equilibrium and of Guo's forcing term;
* decay rate of a shear wave: nu = cs2 (tau - 1/2) (SRT) and
  nu = cs2 (1/s_nu - 1/2) independent of the other MRT rates;
* MRT with every rate 1/tau reduces to SRT;
* conservation of mass and total momentum on a periodic grid;
* square/cube-group symmetry of an unjittered droplet.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import oracle as O
from tests.exact_step import exact_steps
from workload import droplet_rho


def _rand_rational(shape, seed):
    rng = np.random.default_rng(seed)
    vals = rng.integers(20, 120, size=shape)
    return vals, {idx: Fr(int(v), 64) for idx, v in np.ndenumerate(vals)}


def _compare_exact(lattice, shape, order, tau, nsteps, collision="srt", s_bulk=None, s_ghost=None):
    vals, rho_ex = _rand_rational(shape, 11 + order)
    G = -5
    fex = exact_steps(rho_ex, shape, lattice, order, G, Fr(1, 3), tau, nsteps,
                      collision, s_bulk, s_ghost)
    o = O.Oracle(vals / 64.0, lattice, order=order, G=float(G), c0=1.0 / 3.0, psi="identity",
                 tau=float(tau), collision=collision,
                 s_bulk=float(s_bulk or 1.0), s_ghost=float(s_ghost or 1.0))
    o.step(nsteps)
    f = o.get_f()
    ex = np.zeros_like(f)
    for idx in np.ndindex(*shape):
        for q, v in enumerate(fex[idx]):
            ex[(q,) + idx] = float(v)
    # normwise relative error over the whole state
    return np.max(np.abs(f - ex)) / np.max(np.abs(ex))


@pytest.mark.parametrize("order", [4, 6, 8, 10])
@pytest.mark.parametrize("tau", [Fr(1), Fr(4, 5)])
def test_exact_step_d2q9(order, tau):
    assert _compare_exact("D2Q9", (8, 7), order, tau, 2) < 1e-14


@pytest.mark.parametrize("order", [4, 6, 8])
def test_exact_step_d3q19_srt(order):
    assert _compare_exact("D3Q19", (5, 4, 6), order, Fr(6, 5), 1) < 1e-14


@pytest.mark.parametrize("order", [4, 8])
def test_exact_step_d3q19_mrt(order):
    assert _compare_exact("D3Q19", (5, 4, 6), order, Fr(9, 10), 1, "mrt",
                          Fr(11, 10), Fr(13, 10)) < 1e-14


def _unstream(o, f_new):
    """Post-collision values f*(x) = f_new(x + c)."""
    out = np.empty_like(f_new)
    for q, c in enumerate(o.c):
        shift = tuple(-int(ci) for ci in c[:o.dim])
        out[q] = np.roll(f_new[q], shift, axis=tuple(range(o.dim)))
    return out


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (16, 12)), ("D3Q19", (6, 5, 4))])
@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_equilibrium_and_guo_moments(lattice, shape, tau):
    """Post-collision moments: sum f* = rho; sum f* c = sum f c + F (Guo's
    forcing adds the full force per step whatever tau); and at tau = 1,
    sum f* c_i c_j = rho cs2 delta_ij + rho u_i u_j + (u_i F_j + F_i u_j)/2."""
    rng = np.random.default_rng(3)
    rho0 = rng.uniform(0.2, 1.8, shape)
    o = O.Oracle(rho0, lattice, order=4, G=-5.0, tau=tau)
    o.step(3)  # develop a velocity field
    fl = o.fields()
    f0 = o.get_f()
    o.step(1)
    fs = _unstream(o, o.get_f())
    c = o.c[:, :o.dim].astype(float)
    rho, F, u = fl["rho"], fl["F"], fl["u"]
    assert np.allclose(fs.sum(axis=0), rho, rtol=1e-13, atol=0)
    for d in range(o.dim):
        j0 = np.tensordot(c[:, d], f0, axes=1)
        js = np.tensordot(c[:, d], fs, axes=1)
        assert np.allclose(js, j0 + F[d], rtol=0, atol=1e-13)
    if tau == 1.0:
        for i in range(o.dim):
            for j in range(o.dim):
                pij = np.tensordot(c[:, i] * c[:, j], fs, axes=1)
                exp = rho * u[i] * u[j] + 0.5 * (u[i] * F[j] + F[i] * u[j])
                if i == j:
                    exp = exp + rho * o.cs2
                assert np.allclose(pij, exp, rtol=0, atol=1e-13)


def _feq(c, w, cs2, rho, u):
    cu = np.tensordot(c, u, axes=1)
    uu = (u ** 2).sum(axis=0)
    return np.stack([w[q] * rho * (1 + cu[q] / cs2 + cu[q] ** 2 / (2 * cs2 * cs2) - uu / (2 * cs2))
                     for q in range(len(w))])


def _shear_decay(lattice, shape, tau, collision="srt", s_bulk=1.2, s_ghost=1.2, steps=200):
    dim = len(shape)
    o = O.Oracle(np.ones(shape), lattice, order=4, G=0.0, tau=tau, collision=collision,
                 s_bulk=s_bulk, s_ghost=s_ghost)
    ny = shape[1]
    k = 2 * math.pi / ny
    U = 1e-4
    y = np.arange(ny, dtype=float)
    u = np.zeros((dim,) + shape)
    prof = U * np.sin(k * y)
    u[0] = prof.reshape((1, ny) + (1,) * (dim - 2))
    c = o.c[:, :dim].astype(float)
    o.set_f(_feq(c, o.w, o.cs2, np.ones(shape), u))
    amps = []
    for _ in range(2):
        o.step(steps)
        ux = o.fields()["u"][0]
        axes = tuple(a for a in range(dim) if a != 1)
        line = ux.mean(axis=axes)
        amps.append(2.0 / ny * np.dot(line, np.sin(k * y)))
    rate = math.log(amps[0] / amps[1]) / steps
    return rate / (k * k)


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.4])
def test_shear_wave_viscosity_srt(tau):
    nu = _shear_decay("D2Q9", (4, 64), tau)
    assert abs(nu - (tau - 0.5) / 3.0) < 2e-3 * (tau - 0.5) / 3.0


@pytest.mark.parametrize("s_bulk,s_ghost", [(1.2, 1.2), (0.7, 1.9)])
def test_shear_wave_viscosity_mrt(s_bulk, s_ghost):
    tau = 0.9
    nu = _shear_decay("D3Q19", (4, 64, 4), tau, "mrt", s_bulk, s_ghost)
    # the other rates enter only at O(k^2): 0.5% at k = 2 pi / 64
    assert abs(nu - (tau - 0.5) / 3.0) < 5e-3 * (tau - 0.5) / 3.0


def _sound_decay(tau, s_bulk, nx=128, steps=3000):
    """Density amplitude of a standing sound wave rho = 1 + A cos(k x) on an
    nx x 1 x 1 D3Q19 MRT grid without interaction (G = 0), fitted by
    exp(-g t) (C cos(w t) + D sin(w t)); returns (g / k^2, w / k)."""
    from scipy.optimize import curve_fit
    k = 2 * math.pi / nx
    x = np.arange(nx, dtype=float)
    rho0 = (1.0 + 1e-4 * np.cos(k * x)).reshape(nx, 1, 1)
    o = O.Oracle(rho0, "D3Q19", order=4, G=0.0, tau=tau, collision="mrt", s_bulk=s_bulk, s_ghost=1.2)
    t, a = [], []
    for n in range(0, steps + 1, 10):
        if n:
            o.step(10)
        t.append(n)
        a.append(2.0 / nx * np.dot(o.fields()["rho"][:, 0, 0], np.cos(k * x)))
    t, a = np.array(t, dtype=float), np.array(a)
    cs = 1.0 / math.sqrt(3.0)

    def model(t, g, w, C, D):
        return np.exp(-g * t) * (C * np.cos(w * t) + D * np.sin(w * t))

    (g, w, C, D), _ = curve_fit(model, t, a, p0=[0.1 * k * k, cs * k, 1e-4, 0.0])
    assert np.max(np.abs(model(t, g, w, C, D) - a)) < 1e-3 * 1e-4   # the fit describes the run
    return g / (k * k), w / k


@pytest.mark.parametrize("s_bulk", [0.7, 1.2, 1.6])
def test_mrt_bulk_rate_sets_sound_attenuation(s_bulk):
    """Closed form of linear acoustics: a plane sound wave decays at
    Gamma k^2 with Gamma = ((4/3) nu + zeta) / 2, the shear viscosity
    nu = cs2 (tau - 1/2) and the bulk viscosity zeta = (2/3) cs2 (1/s_bulk
    - 1/2) that relaxing the trace of the stress (the c^2 moment) at s_bulk
    gives in 3D; it travels at cs.  A dropped or mis-signed bulk term moves
    Gamma by 20-90% over these rates."""
    tau = 0.9
    gam, speed = _sound_decay(tau, s_bulk)
    nu = (tau - 0.5) / 3.0
    zeta = (2.0 / 3.0) * (1.0 / s_bulk - 0.5) / 3.0
    expect = 0.5 * (4.0 / 3.0 * nu + zeta)
    # lattice corrections are O(k^2): below 1% at k = 2 pi / 128
    assert abs(gam - expect) < 1e-2 * expect, (gam, expect)
    assert abs(speed - 1.0 / math.sqrt(3.0)) < 1e-3


def test_mrt_reduces_to_srt():
    rho0 = droplet_rho((12, 12, 12), 4, seed=3)
    tau = 0.85
    a = O.Oracle(rho0, "D3Q19", order=8, tau=tau, collision="srt").step(20)
    b = O.Oracle(rho0, "D3Q19", order=8, tau=tau, collision="mrt",
                 s_bulk=1 / tau, s_ghost=1 / tau).step(20)
    fa, fb = a.get_f(), b.get_f()
    assert np.max(np.abs(fa - fb)) <= 1e-13 * np.max(np.abs(fa))


@pytest.mark.parametrize("order", [4, 10])
def test_conservation_d2q9(order):
    rho0 = droplet_rho((48, 40), 12, seed=1)
    o = O.Oracle(rho0, "D2Q9", order=order)
    m0 = o.observables()["mass"]
    o.step(2000)
    ob = o.observables()
    assert abs(ob["mass"] - m0) <= 1e-12 * m0  # FP64 rounding drift over the run
    assert np.all(np.abs(ob["mom"]) <= 1e-12 * m0)


def test_conservation_d3q19_mrt():
    rho0 = droplet_rho((16, 14, 12), 4, seed=3)
    o = O.Oracle(rho0, "D3Q19", order=8, collision="mrt")
    m0 = o.observables()["mass"]
    o.step(200)
    ob = o.observables()
    assert abs(ob["mass"] - m0) <= 1e-12 * m0  # FP64 rounding drift over the run
    assert np.all(np.abs(ob["mom"]) <= 1e-12 * m0)


@pytest.mark.parametrize("order", [4, 8])
def test_droplet_symmetry_2d(order):
    rho0 = droplet_rho((32, 32), 9)
    o = O.Oracle(rho0, "D2Q9", order=order).step(300)
    r = o.fields()["rho"]
    # reflections about the centre node 16 and the diagonal
    rx = np.roll(r[::-1, :], 1, axis=0)
    ry = np.roll(r[:, ::-1], 1, axis=1)
    for other in (rx, ry, r.T):
        assert np.max(np.abs(r - other)) <= 1e-12


def test_droplet_symmetry_3d():
    rho0 = droplet_rho((16, 16, 16), 5)
    o = O.Oracle(rho0, "D3Q19", order=8, collision="mrt").step(60)
    r = o.fields()["rho"]
    rx = np.roll(r[::-1], 1, axis=0)
    for other in (rx, r.transpose(1, 0, 2), r.transpose(2, 1, 0)):
        assert np.max(np.abs(r - other)) <= 1e-12
