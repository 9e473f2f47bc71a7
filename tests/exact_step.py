"""Exact-rational brute-force time step (pure Python fractions).

A second, independent statement of one time step of the forced lattice
Boltzmann equation (Sec. 2, Eq. (1), (3), (4)), used to pin the FP64 oracle
on tiny grids with psi = rho and rational inputs.  It is written the other
way round from the oracle: nodes are coordinate tuples in dicts, streaming
pushes each post-collision value to its destination, and MRT is applied as
a sum of rank-one projectors P_k = m_k m_k^T / |m_k|^2 over the orthogonal
moment rows instead of the M, M^-1 pair.
"""
from fractions import Fraction as Fr
from itertools import product

from oracle import tables as T


def _add(a, b, shape):
    return tuple((x + y) % n for x, y, n in zip(a, b, shape))


def exact_steps(rho0, shape, lattice, order, G, c0, tau, nsteps=1,
                collision="srt", s_bulk=None, s_ghost=None, forcing="guo", solid=(), rho_w=None,
                init="equilibrium"):
    """rho0: dict node -> Fraction.  Returns dict node -> list of f (Fractions)
    after nsteps, with f = feq(rho0, 0) at t = 0, or with init == "rest"
    f = feq(rho0, v), v = -F / (2 rho0) and F the force of psi = rho0 on
    the periodic grid (walls play no part in the start).

    solid: nodes of a wall (initialised like the rest).  In the force they count with
    psi = rho_w (the virtual wall density, Sec. 3); in place of a collision
    they send every population back the way it came (standard bounce-back)."""
    dim, cs2, vel = T.lattice(lattice)
    stencil = T.force_stencil(dim, order)
    tau = Fr(tau)
    G, c0 = Fr(G), Fr(c0)
    nodes = list(product(*[range(n) for n in shape]))
    solid = set(solid)
    back = {q: [tuple(-v for v in c) for c, _ in vel].index(tuple(c)) for q, (c, _) in enumerate(vel)}
    f = {x: [w * rho0[x] for _, w in vel] for x in nodes}
    if init == "rest":
        for x in nodes:
            acc = [Fr(0)] * dim
            for e, w in stencil:
                pn = rho0[_add(x, e, shape)]
                for d in range(dim):
                    acc[d] += w * pn * e[d]
            v = [G * c0 * rho0[x] * a / (2 * rho0[x]) for a in acc]   # -F / (2 rho)
            vv = sum(a * a for a in v)
            f[x] = []
            for c, w in vel:
                cv = sum(c[d] * v[d] for d in range(dim))
                f[x].append(w * rho0[x] * (1 + cv / cs2 + cv * cv / (2 * cs2 * cs2) - vv / (2 * cs2)))
    elif init != "equilibrium":
        raise ValueError(init)
    if collision == "mrt":
        rows, groups = T.mrt_gram_schmidt(lattice)
        rate = {}
        for k in groups["cons"]:
            rate[k] = Fr(0)
        for k in groups["bulk"]:
            rate[k] = Fr(s_bulk)
        for k in groups["shear"]:
            rate[k] = 1 / tau
        for k in groups["ghost"]:
            rate[k] = Fr(s_ghost)
        norms = [sum(v * v for v in r) for r in rows]

    for _ in range(nsteps):
        rho = {x: sum(f[x]) for x in nodes}
        # psi = rho (identity) keeps everything rational; walls carry rho_w
        psi = {x: (Fr(rho_w) if x in solid else rho[x]) for x in nodes}
        F = {}
        for x in nodes:
            acc = [Fr(0)] * dim
            for e, w in stencil:
                pn = psi[_add(x, e, shape)]
                for d in range(dim):
                    acc[d] += w * pn * e[d]
            F[x] = [-G * c0 * psi[x] * a for a in acc]
        new = {x: [None] * len(vel) for x in nodes}
        for x in nodes:
            fx = f[x]
            if x in solid:
                # population q leaves along c_q what arrived along -c_q
                for q, (c, _) in enumerate(vel):
                    new[_add(x, c, shape)][q] = fx[back[q]]
                continue
            mom = [sum(fb * c[d] for fb, (c, _) in zip(fx, vel)) for d in range(dim)]
            u = [(mom[d] + F[x][d] / 2) / rho[x] for d in range(dim)]
            uu = sum(ui * ui for ui in u)
            feq, ph = [], []
            for c, w in vel:
                cu = sum(c[d] * u[d] for d in range(dim))
                feq.append(rho[x] * w * (1 + cu / cs2 + cu * cu / (2 * cs2 * cs2) - uu / (2 * cs2)))
                ph.append(w * sum(((c[d] - u[d]) / cs2 + cu * c[d] / (cs2 * cs2)) * F[x][d]
                                  for d in range(dim)))
            if forcing == "edm":
                # exact difference method: equilibria at v = mom/rho and v + F/rho
                v = [m / rho[x] for m in mom]
                v2 = [v[d] + F[x][d] / rho[x] for d in range(dim)]

                def eq(vel):
                    vv = sum(t * t for t in vel)
                    out = []
                    for c, w in T.lattice(lattice)[2]:
                        cv = sum(c[d] * vel[d] for d in range(dim))
                        out.append(rho[x] * w * (1 + cv / cs2 + cv * cv / (2 * cs2 * cs2) - vv / (2 * cs2)))
                    return out
                e1, e2 = eq(v), eq(v2)
                fs = [fb - (fb - a) / tau + (b - a) for fb, a, b in zip(fx, e1, e2)]
            elif collision == "srt":
                fs = [fb - (fb - fe) / tau + (1 - 1 / (2 * tau)) * p
                      for fb, fe, p in zip(fx, feq, ph)]
            else:
                fs = list(fx)
                neq = [fb - fe for fb, fe in zip(fx, feq)]
                for k, r in enumerate(rows):
                    a = sum(rv * v for rv, v in zip(r, neq)) / norms[k]
                    b = sum(rv * v for rv, v in zip(r, ph)) / norms[k]
                    coeff = -rate[k] * a + (1 - rate[k] / 2) * b
                    for q in range(len(fs)):
                        fs[q] += coeff * r[q]
            for q, (c, _) in enumerate(vel):
                new[_add(x, c, shape)][q] = fs[q]
        f = new
    return f
