"""Pins for the oracle's lattice and force-stencil tables.

Everything here is exact (fractions) except the last checks, which compare
the C oracle's double tables with the exact ones to one rounding.
"""
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import oracle as O
from oracle import tables as T

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def table1():
    rows = {}
    for line in open(GOLD):
        line = line.split("#")[0].split()
        if not line:
            continue
        name, cs2 = line[0], Fr(line[1])
        rows[name] = (cs2, {int(k): Fr(v) for k, v in (t.split(":") for t in line[2:])})
    return rows


def test_table1_golden_matches_lattices():
    gold = table1()
    assert set(gold) == {"D2Q9", "D2Q13", "D2Q25"}
    for name, (cs2, w) in gold.items():
        dim, lcs2, wmap = T.LATTICE_WEIGHTS[name]
        assert lcs2 == cs2
        assert wmap == w


@pytest.mark.parametrize("name", ["D2Q9", "D2Q13", "D2Q25", "D3Q19"])
def test_lattice_moments(name):
    """sum w = 1, sum w c_x^2 = cs2, sum w c_x^2 c_y^2 = cs2^2 (the Hermite
    conditions that make Eq. (4)'s equilibrium reproduce the pressure tensor)."""
    dim, cs2, vel = T.lattice(name)
    z = (0,) * (dim - 2)
    assert sum(w for _, w in vel) == 1
    assert T.moment(vel, (2, 0) + z) == cs2
    assert T.moment(vel, (2, 2) + z) == cs2 ** 2
    assert T.moment(vel, (4, 0) + z) == 3 * cs2 ** 2
    assert T.moment(vel, (1, 0) + z) == 0


@pytest.mark.parametrize("name,order", [("D2Q9", 4), ("D2Q13", 6), ("D2Q25", 8), ("D3Q19", 4)])
def test_lattice_isotropy_order(name, order):
    """Sec. 3: nearest-neighbour sets (D2Q9, D3Q19) reach only 4th-order
    isotropy; D2Q13 and D2Q25 reach 6th and 8th."""
    dim, cs2, vel = T.lattice(name)
    assert T.isotropy_order(vel, dim) == order


def test_equal_viscosity_taus():
    """Sec. 3: tau = 11/12 (D2Q13) and 19/24 (D2Q25) give the viscosity of
    D2Q9 at tau = 1, nu = cs2 (tau - 1/2)."""
    nu9 = Fr(1, 3) * (1 - Fr(1, 2))
    assert T.LATTICE_WEIGHTS["D2Q13"][1] * (Fr(11, 12) - Fr(1, 2)) == nu9
    assert T.LATTICE_WEIGHTS["D2Q25"][1] * (Fr(19, 24) - Fr(1, 2)) == nu9


@pytest.mark.parametrize("dim,order", sorted(T.FORCE_SHELLS))
def test_force_stencil_isotropy(dim, order):
    vecs = T.force_stencil(dim, order)
    assert T.moment(vecs, (2,) + (0,) * (dim - 1)) == 1
    assert T.isotropy_order(vecs, dim) == order
    assert all(w > 0 for _, w in vecs)


def test_force_stencils_match_table1():
    """The D2Q13 and D2Q25 non-rest weights of Table 1 are the E6 and E8
    force weights scaled by their cs2 (2/5 and 4/7); E4 is the classic
    nearest-neighbour pair 1/3, 1/12."""
    gold = table1()
    e6, e8 = T.force_weights(2, 6), T.force_weights(2, 8)
    cs2, w13 = gold["D2Q13"]
    assert {k: v for k, v in w13.items() if k} == {k: cs2 * v for k, v in e6.items()}
    cs2, w25 = gold["D2Q25"]
    assert {k: v for k, v in w25.items() if k} == {k: cs2 * v for k, v in e8.items()}
    assert T.force_weights(2, 4) == {1: Fr(1, 3), 2: Fr(1, 12)}


def test_force_stencil_sizes_and_radius():
    sizes = {(2, 4): 8, (2, 6): 12, (2, 8): 24, (2, 10): 36, (3, 4): 18, (3, 6): 32, (3, 8): 92}
    radius = {(2, 4): 1, (2, 6): 2, (2, 8): 2, (2, 10): 3, (3, 4): 1, (3, 6): 2, (3, 8): 2}
    for key in sizes:
        assert len(T.force_stencil(*key)) == sizes[key]
        assert T.stencil_radius(*key) == radius[key]


def test_taylor_coefficients_isotropic_terms():
    """a_1 = lambda_4 / 2 with lambda_4 = sum w e_x^2 e_y^2: 1/3, 2/5, 4/7, 12/17
    for E4/6/8/10 (the rank-4 coefficient)."""
    lam4 = {4: Fr(1, 3), 6: Fr(2, 5), 8: Fr(4, 7), 10: Fr(12, 17)}
    for order, lam in lam4.items():
        vecs = T.force_stencil(2, order)
        assert T.moment(vecs, (2, 2)) == lam
        assert T.taylor_coefficients(2, order)[1] == lam / 2


@pytest.mark.parametrize("name", ["D2Q9", "D2Q13", "D2Q25", "D3Q19"])
def test_c_oracle_lattice_tables(name):
    dim, c, w, cs2 = O.lattice_table(name)
    edim, ecs2, vel = T.lattice(name)
    assert dim == edim and cs2 == float(ecs2)
    got = sorted((tuple(int(x) for x in ci[:dim]), wi) for ci, wi in zip(c, w))
    exp = sorted((tuple(ci), float(wi)) for ci, wi in vel)
    assert len(got) == len(exp)
    for (cg, wg), (ce, we) in zip(got, exp):
        assert cg == ce and abs(wg - we) <= 1e-16 * we


@pytest.mark.parametrize("dim,order", sorted(T.FORCE_SHELLS))
def test_c_oracle_stencil_tables(dim, order):
    e, w = O.stencil_table(dim, order)
    got = sorted((tuple(int(x) for x in ei[:dim]), wi) for ei, wi in zip(e, w))
    exp = sorted((tuple(ei), float(wi)) for ei, wi in T.force_stencil(dim, order))
    assert len(got) == len(exp)
    for (eg, wg), (ee, we) in zip(got, exp):
        assert eg == ee and abs(wg - we) <= 1e-16 * we


def test_mrt_basis_orthogonal_and_matches_c():
    rows, groups = T.mrt_gram_schmidt("D3Q19")
    n = len(rows)
    for i in range(n):
        for j in range(i):
            assert sum(a * b for a, b in zip(rows[i], rows[j])) == 0
    rho0 = np.ones((4, 4, 4))
    o = O.Oracle(rho0, "D3Q19", order=4, collision="mrt", s_bulk=1.1, s_ghost=1.3, tau=0.8)
    M, nn, S = o.mrt_basis()
    # the C oracle enumerates velocities in the same shell/lexicographic order
    _, c, _, _ = O.lattice_table("D3Q19")
    dim, _, vel = T.lattice("D3Q19")
    assert [tuple(v) for v in c] == [tuple(v) for v, _ in vel]
    ex = np.array([[float(x) for x in r] for r in rows])
    assert np.allclose(M, ex, atol=1e-13, rtol=0)
    assert np.allclose(nn, (ex ** 2).sum(axis=1), rtol=1e-14)
    exp_S = np.zeros(19)
    exp_S[groups["bulk"]] = 1.1
    exp_S[groups["shear"]] = 1 / 0.8
    exp_S[groups["ghost"]] = 1.3
    assert np.allclose(S, exp_S, rtol=1e-15)
