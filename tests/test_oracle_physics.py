"""Physics pins of the oracle: flat interface (Sec. 3, coexistence test) and
the Laplace law for droplets (Sec. 3, droplet test; p from the psi
definition of Sec. 3).

Flat interface.  Along a 1D interface the transverse force and velocity
vanish identically.  The bulk densities are fixed by mechanical balance:
p(rho_v) = p(rho_l) = p0 with p = cs2 rho + G c0 psi^2 / 2 and an
equal-area condition int (p0 - p) psi'/psi^(1+eps) d rho = 0.  For the
Guo-forced model with the nearest-neighbour (E4) stencil the discrete
balance is the eps = 0 member of this family (Li, Luo & Li, Phys. Rev. E 86,
016709 (2012) analyse this family of conditions); the continuum Taylor
argument gives eps = 1.  The densities must also be independent of tau.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import fsolve

from oracle import oracle as O
from workload import droplet_rho, slab_rho

CS2, GC0 = 1.0 / 3.0, -5.0 / 3.0


def _psi(r):
    return 1.0 - np.exp(-r)


def _p(r):
    return CS2 * r + 0.5 * GC0 * _psi(r) ** 2


def equal_area(eps):
    def eqs(v):
        rv, rl = v
        p0 = _p(rl)
        integ = quad(lambda r: (p0 - _p(r)) * np.exp(-r) / _psi(r) ** (1 + eps), rv, rl,
                     epsabs=1e-14, epsrel=1e-12)[0]
        return [_p(rv) - _p(rl), integ]
    return fsolve(eqs, [0.15, 1.9], xtol=1e-13)


@pytest.fixture(scope="module")
def slabs():
    out = {}
    for tau in (0.7, 1.0, 1.5):
        o = O.Oracle(slab_rho((64, 4), 32), "D2Q9", order=4, tau=tau)
        o.step(15000)
        out[tau] = o.fields()
    return out


def test_flat_interface_transverse_zero(slabs):
    fl = slabs[1.0]
    assert np.max(np.abs(fl["F"][1])) == 0.0
    assert np.max(np.abs(fl["u"][1])) == 0.0
    r = fl["rho"][:, 0]
    # mirror symmetry of the slab about its centre node 32
    assert np.max(np.abs(r - np.roll(r[::-1], 1))) < 1e-10


def test_flat_interface_coexistence_e4(slabs):
    rv, rl = equal_area(0.0)
    for tau, fl in slabs.items():
        r = fl["rho"][:, 0]
        assert abs(r.max() - rl) < 2e-5 * rl, (tau, r.max(), rl)
        assert abs(r.min() - rv) < 2e-5 * rv, (tau, r.min(), rv)


def test_flat_interface_tau_independent(slabs):
    """Bulk densities do not depend on tau (tau = 0.7 relaxes more slowly, so
    its interface profile is compared only in the bulk)."""
    ref = slabs[1.0]["rho"][:, 0]
    for tau in (0.7, 1.5):
        r = slabs[tau]["rho"][:, 0]
        assert abs(r.max() - ref.max()) < 1e-5 * ref.max()
        assert abs(r.min() - ref.min()) < 1e-5 * ref.min()
    assert np.max(np.abs(slabs[1.5]["rho"][:, 0] - ref)) < 1e-8


def test_flat_interface_not_continuum_rule(slabs):
    """The continuum eps = 1 rule is visibly different (more than 10% in the
    vapour density), so the eps = 0 match above is not an accident."""
    rv1, _ = equal_area(1.0)
    rmin = slabs[1.0]["rho"][:, 0].min()
    assert abs(rmin - rv1) > 0.1 * rv1


def test_laplace_law():
    """dp = sigma / R in 2D: linear in 1/R_eq with a small intercept."""
    rs, dps = [], []
    for R in (10, 13, 16, 20):
        o = O.Oracle(droplet_rho((64, 64), R), "D2Q9", order=4)
        o.step(4000)
        ob = o.observables()
        rs.append(ob["radius"])
        dps.append(ob["dp"])
    rs, dps = np.array(rs), np.array(dps)
    A = np.vstack([1.0 / rs, np.ones_like(rs)]).T
    coef = np.linalg.lstsq(A, dps, rcond=None)[0]
    pred = A @ coef
    r2 = 1.0 - ((dps - pred) ** 2).sum() / ((dps - dps.mean()) ** 2).sum()
    assert r2 > 0.999
    assert coef[0] > 0
    assert abs(coef[1]) < 0.1 * dps.min()


def test_spurious_currents_fall_modestly_with_force_isotropy():
    """Sec. 2: raising the isotropy order of the force stencil alone (Shan's
    remedy) lowers the spurious currents, but only partly, because the
    velocity set's own tensors stay at their order.  The oracle's 256^2
    droplet (tests/golden/droplet_256_orders_oracle.json, 50,000 steps) shows
    both: max|u| falls with every order E4 -> E6 -> E8 -> E10, yet E10 keeps
    more than a tenth of the E4 value; the Laplace jump stays within a
    factor 2 across the orders (the bulk state changes little)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "droplet_256_orders_oracle.json")
    with open(path) as fh:
        g = json.load(fh)["orders"]
    umax = [g[o]["traj"][-1]["max_u"] for o in ("4", "6", "8", "10")]
    dp = [g[o]["traj"][-1]["dp"] for o in ("4", "6", "8", "10")]
    assert all(a > b for a, b in zip(umax, umax[1:])), umax
    assert umax[-1] > 0.1 * umax[0], umax
    assert max(dp) < 2.0 * min(dp), dp
