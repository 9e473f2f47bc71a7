"""Peng-Robinson equation of state of the paper's experiments (Sec. 3), for
setting up runs of the library: the EOS parameters at a reduced temperature
and the Maxwell coexistence densities that seed the initial profile.

    p(rho) = rho R T / (1 - b rho) - a alpha(T) rho^2 / (1 + 2 b rho - b^2 rho^2)
    alpha(T) = [1 + kappa (1 - sqrt(T / Tc))]^2,
    kappa = 0.37464 + 1.54226 omega - 0.26992 omega^2,
with a = 2/49, b = 2/21, R = 1, omega = 0.344 (Sec. 3).

The critical point is located from its definition with alpha = 1: writing
p = rho R T / (1 - b rho) - a g(rho), g = rho^2 / (1 + 2 b rho - b^2 rho^2),
dp/drho = 0 gives R T = a g'(rho) (1 - b rho)^2 and d2p/drho2 = 0 gives
2 b R T = a g''(rho) (1 - b rho)^3; eliminating T leaves the one-variable
equation 2 b g'(rho) = g''(rho) (1 - b rho), solved by bisection.
"""
import math

A, B, RGAS, OMEGA = 2.0 / 49.0, 2.0 / 21.0, 1.0, 0.344


def _g1(r, b):
    """g'(rho) of g = rho^2 / (1 + 2 b rho - b^2 rho^2)."""
    d = 1.0 + 2.0 * b * r - b * b * r * r
    return (2.0 * r * d - r * r * (2.0 * b - 2.0 * b * b * r)) / (d * d)


def _g2(r, b, h=1e-6):
    return (_g1(r + h, b) - _g1(r - h, b)) / (2.0 * h)


def _bisect(f, lo, hi, iters=200):
    flo = f(lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if (fm < 0) == (flo < 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def critical_point(a=A, b=B, R=RGAS):
    """(Tc, rho_c) of the Peng-Robinson EOS (alpha = 1)."""
    f = lambda r: 2.0 * b * _g1(r, b) - _g2(r, b) * (1.0 - b * r)  # noqa: E731
    # the root lies well inside (0, 1/b); scan for the sign change first
    xs = [k / 400.0 / b for k in range(1, 400)]
    for x0, x1 in zip(xs, xs[1:]):
        if (f(x0) < 0) != (f(x1) < 0):
            rc = _bisect(f, x0, x1)
            return a * _g1(rc, b) * (1.0 - b * rc) ** 2 / R, rc
    raise RuntimeError("no critical point")


def kappa(omega=OMEGA):
    return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega


def params_at(Tr, omega=OMEGA, a=A, b=B, R=RGAS):
    """EOS fields for the library (eos= of make_params / Sim) at T = Tr Tc."""
    Tc, _ = critical_point(a, b, R)
    alpha = (1.0 + kappa(omega) * (1.0 - math.sqrt(Tr))) ** 2
    return {"a": a, "b": b, "R": R, "T": Tr * Tc, "alpha": alpha}


def pressure(rho, eos):
    br = eos["b"] * rho
    return rho * eos["R"] * eos["T"] / (1.0 - br) - eos["a"] * eos["alpha"] * rho * rho / (1.0 + 2.0 * br - br * br)


def maxwell(eos, n=4000):
    """(rho_v, rho_l) from the equal-area rule in the specific volume:
    p(rho_v) = p(rho_l) = p0 and int_{v_l}^{v_v} (p - p0) dv = 0, v = 1/rho."""
    b = eos["b"]
    p = lambda r: pressure(r, eos)  # noqa: E731
    dp = lambda r: (p(r * (1 + 1e-7)) - p(r * (1 - 1e-7))) / (2e-7 * r)  # noqa: E731
    # spinodals: the local maximum and minimum of p(rho)
    xs = [(k + 0.5) / n * 0.999 / b for k in range(n)]
    ext = []
    for x0, x1 in zip(xs, xs[1:]):
        if (dp(x0) < 0) != (dp(x1) < 0):
            ext.append(_bisect(dp, x0, x1, 100))
    if len(ext) < 2:
        raise ValueError("no two-phase region at this temperature")
    s1, s2 = ext[0], ext[1]
    hi = 0.999 / b

    def roots(p0):
        # p(0) = 0 < p0: the vapour root is bracketed from rho = 0
        return (_bisect(lambda r: p(r) - p0, 0.0, s1, 200), _bisect(lambda r: p(r) - p0, s2, hi, 200))

    def area(p0, m=4000):
        rv, rl = roots(p0)
        # int (p - p0) dv over v in [1/rl, 1/rv] = int (p - p0) v d(ln v),
        # composite Simpson in ln v (the vapour volume spans decades)
        t0, t1 = -math.log(rl), -math.log(rv)
        h = (t1 - t0) / m
        s = 0.0
        for k in range(m + 1):
            v = math.exp(t0 + k * h)
            wk = 1 if k in (0, m) else (4 if k % 2 else 2)
            s += wk * (p(1.0 / v) - p0) * v
        return s * h / 3.0

    lo, hi_p = max(p(s2), 1e-14) * (1 + 1e-12), p(s1) * (1 - 1e-12)
    if area(lo) * area(hi_p) > 0:
        raise ValueError("no equal-area root at a positive pressure")
    p0 = _bisect(area, lo, hi_p, 80)
    return roots(p0)
