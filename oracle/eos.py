"""Peng-Robinson equation of state for the pseudo-potential (Sec. 3).

TEST INFRASTRUCTURE (oracle side): used by tests/ only.

    p(rho) = rho R T / (1 - b rho) - a alpha(T) rho^2 / (1 + 2 b rho - b^2 rho^2)
    alpha(T) = [1 + kappa (1 - sqrt(T / Tc))]^2,
    kappa = 0.37464 + 1.54226 omega - 0.26992 omega^2,
with a = 2/49, b = 2/21, R = 1 and omega = 0.344 in the droplet tests of
Sec. 3.  The critical temperature is found here from its definition
(dp/drho = d2p/drho2 = 0 at alpha = 1), not from tabulated constants.

The pseudo-potential follows from p = cs2 rho + G c0 psi^2 / 2 (Sec. 3, with
cs'^2 = c0 for the normalised force weights):
    psi = sqrt(2 (p - cs2 rho) / (G c0)).
"""
import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq, fsolve

A, B, RGAS, OMEGA = 2.0 / 49.0, 2.0 / 21.0, 1.0, 0.344


def pressure(rho, T, alpha, a=A, b=B, R=RGAS):
    return rho * R * T / (1.0 - b * rho) - a * alpha * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho)


def kappa(omega=OMEGA):
    return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega


def critical_point(a=A, b=B, R=RGAS):
    """(Tc, rho_c) from dp/drho = 0 and d2p/drho2 = 0 with alpha = 1, both
    derivatives written out: with D = 1 + 2 b rho - b^2 rho^2,
        dp/drho   = R T / (1 - b rho)^2 - 2 a rho (1 + b rho) / D^2
        d2p/drho2 = 2 b R T / (1 - b rho)^3
                    - 2 a [(1 + 2 b rho) D - 4 rho (1 + b rho)(b - b^2 rho)] / D^3."""
    def eqs(v):
        T, rho = v
        D = 1.0 + 2.0 * b * rho - b * b * rho * rho
        d1 = R * T / (1.0 - b * rho) ** 2 - 2.0 * a * rho * (1.0 + b * rho) / D ** 2
        d2 = (2.0 * b * R * T / (1.0 - b * rho) ** 3
              - 2.0 * a * ((1.0 + 2.0 * b * rho) * D - 4.0 * rho * (1.0 + b * rho) * (b - b * b * rho)) / D ** 3)
        return [d1, d2]

    sol = fsolve(eqs, [0.07, 2.5], xtol=1e-14)
    return float(sol[0]), float(sol[1])


def alpha(T, Tc, omega=OMEGA):
    return (1.0 + kappa(omega) * (1.0 - np.sqrt(T / Tc))) ** 2


def eos_params(Tr, omega=OMEGA, a=A, b=B, R=RGAS):
    """Oracle/library EOS parameter dict at reduced temperature Tr = T/Tc."""
    Tc, _ = critical_point(a, b, R)
    T = Tr * Tc
    return {"a": a, "b": b, "R": R, "T": T, "alpha": float(alpha(T, Tc, omega)), "Tc": Tc, "omega": omega}


def psi(rho, eos, cs2, G, c0):
    arg = 2.0 * (pressure(rho, eos["T"], eos["alpha"], eos["a"], eos["b"], eos["R"]) - cs2 * rho) / (G * c0)
    return np.sqrt(np.maximum(arg, 0.0))


def _p_of(eos):
    return lambda r: pressure(r, eos["T"], eos["alpha"], eos["a"], eos["b"], eos["R"])


def spinodals(eos, lo=1e-4, hi=None):
    """(rho_s1, rho_s2): the local maximum and minimum of p(rho) (T < Tc)."""
    p = _p_of(eos)
    hi = hi or 0.999 / eos["b"]
    x = np.linspace(lo, hi, 200001)
    d = np.gradient(p(x), x)
    idx = np.where(np.diff(np.sign(d)) != 0)[0]
    roots = [brentq(lambda r: (p(r + 1e-7) - p(r - 1e-7)) / 2e-7, x[i], x[i + 1]) for i in idx[:2]]
    return roots[0], roots[1]


def _outer_roots(p, p0, s1, s2, hi):
    rv = brentq(lambda r: p(r) - p0, 0.0, s1)
    rl = brentq(lambda r: p(r) - p0, s2, hi)
    return rv, rl


def _coexistence(eos, weight):
    """Solve p(rho_v) = p(rho_l) = p0 with int_{rho_v}^{rho_l} (p - p0) weight drho = 0."""
    p = _p_of(eos)
    s1, s2 = spinodals(eos)
    hi = 0.999 / eos["b"]
    pmax, pmin = p(s1), max(p(s2), 1e-12)

    def area(p0):
        rv, rl = _outer_roots(p, p0, s1, s2, hi)
        return quad(lambda r: (p(r) - p0) * weight(r), rv, rl, epsabs=1e-14, epsrel=1e-12, limit=200)[0]

    eps = 1e-12 * pmax
    a_lo, a_hi = area(pmin + eps), area(pmax - eps)
    if a_lo * a_hi > 0:
        return None   # no coexistence at a positive pressure for this rule
    p0 = brentq(area, pmin + eps, pmax - eps, xtol=1e-15)
    return _outer_roots(p, p0, s1, s2, hi)


def maxwell(eos):
    """Coexistence (rho_v, rho_l) of the EOS by the equal-area rule in the
    specific volume 1/rho: int (p - p0) d(1/rho) = 0."""
    return _coexistence(eos, lambda r: 1.0 / (r * r))


def mechanical(eos, cs2, G, c0, eps=0.0):
    """Coexistence from p(rho_v) = p(rho_l) = p0 and
    int (p0 - p) psi'/psi^(1+eps) drho = 0 (psi of the pseudo-potential)."""
    ps = lambda r: psi(r, eos, cs2, G, c0)  # noqa: E731

    def wgt(r, h=1e-7):
        return (ps(r + h) - ps(r - h)) / (2 * h) / ps(r) ** (1 + eps)
    return _coexistence(eos, wgt)
