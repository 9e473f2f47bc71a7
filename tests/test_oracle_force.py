"""Pins for the oracle's interaction-force operator (Sec. 2, Eq. (1)-(2)).

* plane wave: for psi = cos(k.x), sum_a w_a psi(x+e_a) e_a = -sin(k.x) S(k)
  with S(k) = sum_a w_a e_a sin(k.e_a) (the cosine part cancels between
  +e and -e), so F = G c0 cos(k.x) sin(k.x) S(k) exactly;
* Taylor (Eq. (2)): on a smooth field, F / (-G c0 psi) matches
  sum_m a_m d_i lap^m psi with a_0 = 1, and the remainder after the terms
  whose tensors are isotropic falls like k^(order+1);
* periodic invariant: sum_x F(x) = 0 (each pair x, x+e cancels).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import tables as T

G, C0 = -5.0, 1.0 / 3.0


def _grid(shape):
    return np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")


@pytest.mark.parametrize("dim,order", sorted(T.FORCE_SHELLS))
def test_plane_wave_closed_form(dim, order):
    shape = (24, 20) if dim == 2 else (12, 10, 8)
    m = (3, 2) if dim == 2 else (2, 1, 3)
    k = np.array([2 * math.pi * mi / n for mi, n in zip(m, shape)])
    X = _grid(shape)
    phase = sum(ki * xi for ki, xi in zip(k, X))
    psi = np.cos(phase)
    lattice = "D2Q9" if dim == 2 else "D3Q19"
    F = O.force(psi, lattice, order, G, C0)
    S = np.zeros(dim)
    for e, w in T.force_stencil(dim, order):
        S += float(w) * np.array(e, dtype=float) * math.sin(float(np.dot(k, e)))
    for d in range(dim):
        exact = G * C0 * np.cos(phase) * np.sin(phase) * S[d]
        assert np.max(np.abs(F[d] - exact)) <= 1e-13 * max(1.0, np.max(np.abs(exact)))


@pytest.mark.parametrize("order", [4, 6, 8, 10])
def test_taylor_remainder_order_2d(order):
    """Oblique plane wave of shrinking k: remainder after the isotropic
    Taylor terms scales as k^(order+1) (slope within 0.15)."""
    coef = [float(a) for a in T.taylor_coefficients(2, order)]
    theta = math.pi / 8
    errs = []
    ks = [0.4, 0.2] if order < 10 else [0.8, 0.4]
    for kmag in ks:
        k = kmag * np.array([math.cos(theta), math.sin(theta)])
        # plane wave on the lattice: use exact sum instead of a periodic grid
        # (k is not commensurate); evaluate at x = 0 with psi = sin(k.x) + 2
        s = np.zeros(2)
        for e, w in T.force_stencil(2, order):
            s += float(w) * np.array(e, dtype=float) * (math.sin(float(np.dot(k, e))) + 2.0)
        # d_i lap^m psi at x=0 for psi = sin(k.x): k_i (-|k|^2)^m cos(0)
        taylor = sum(a * (-kmag ** 2) ** m for m, a in enumerate(coef)) * k
        errs.append(np.linalg.norm(s - taylor))
    slope = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert abs(slope - (order + 1)) < 0.15


@pytest.mark.parametrize("order", [4, 6, 8, 10])
def test_taylor_leading_term_on_grid(order):
    """F -> -G c0 psi grad(psi) on a smooth periodic field as the grid is
    refined (error ratio 4 per halving of k: the k^3 term)."""
    errs = []
    for n in (32, 64):
        X = _grid((n, n))
        kx, ky = 2 * math.pi / n, 4 * math.pi / n
        psi = 1.0 + 0.3 * np.sin(kx * X[0]) * np.cos(ky * X[1])
        gx = 0.3 * kx * np.cos(kx * X[0]) * np.cos(ky * X[1])
        gy = -0.3 * ky * np.sin(kx * X[0]) * np.sin(ky * X[1])
        F = O.force(psi, "D2Q9", order, G, C0)
        lead = np.stack([-G * C0 * psi * gx, -G * C0 * psi * gy])
        errs.append(np.max(np.abs(F - lead)))
    ratio = errs[0] / errs[1]
    assert 7.0 < ratio < 9.0, ratio


def test_taylor_leading_term_on_grid_3d():
    errs = []
    for n in (16, 32):
        X = _grid((n, n, n))
        k = 2 * math.pi / n
        psi = 1.0 + 0.2 * np.sin(k * X[0] + 2 * k * X[1]) * np.cos(k * X[2])
        g = [0.2 * k * np.cos(k * X[0] + 2 * k * X[1]) * np.cos(k * X[2]),
             0.4 * k * np.cos(k * X[0] + 2 * k * X[1]) * np.cos(k * X[2]),
             -0.2 * k * np.sin(k * X[0] + 2 * k * X[1]) * np.sin(k * X[2])]
        for order in (4, 8):
            F = O.force(psi, "D3Q19", order, G, C0)
            lead = np.stack([-G * C0 * psi * gi for gi in g])
            errs.append(np.max(np.abs(F - lead)))
    for a, b in zip(errs[:2], errs[2:]):
        assert 7.0 < a / b < 9.0


@pytest.mark.parametrize("dim,order", sorted(T.FORCE_SHELLS))
def test_force_sums_to_zero(dim, order):
    rng = np.random.default_rng(5)
    shape = (13, 11) if dim == 2 else (7, 6, 5)
    psi = rng.uniform(0.1, 1.0, shape)
    F = O.force(psi, "D2Q9" if dim == 2 else "D3Q19", order, G, C0)
    for d in range(dim):
        assert abs(F[d].sum()) <= 1e-13 * np.abs(F[d]).sum()


def test_force_brute_force_single_node():
    """Direct evaluation of Eq. (1) at one node of a random field, with the
    stencil vectors written out by hand for E4 in 2D."""
    rng = np.random.default_rng(7)
    psi = rng.uniform(0.2, 1.0, (9, 7))
    F = O.force(psi, "D2Q9", 4, G, C0)
    x, y = 0, 6
    acc = np.zeros(2)
    for ex, ey, w in [(1, 0, 1 / 3), (-1, 0, 1 / 3), (0, 1, 1 / 3), (0, -1, 1 / 3),
                      (1, 1, 1 / 12), (1, -1, 1 / 12), (-1, 1, 1 / 12), (-1, -1, 1 / 12)]:
        acc += w * psi[(x + ex) % 9, (y + ey) % 7] * np.array([ex, ey])
    exp = -G * C0 * psi[x, y] * acc
    assert np.allclose(F[:, x, y], exp, rtol=1e-14, atol=0)
