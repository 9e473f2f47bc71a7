"""Exact-rational lattice and force-stencil tables for the FP64 oracle.

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the CPU-baseline
leg of bench.py may import anything under oracle/. The GPU library carries its
own constants and never reads this module.

Two families of tables, both kept as fractions.Fraction:

* LB velocity sets c_beta with weights w_beta and sound speed c_s^2
  (Sec. 3, Table 1 for D2Q9, D2Q13, D2Q25; D3Q19 is the standard nearest-
  neighbour cube lattice that Sec. 3 names among the 4th-order-isotropic ones).
* Interaction-force stencils e_alpha with normalised weights w_hat(|e|^2)
  (Sec. 2, Eq. (1) and the isotropy argument around Eq. (2)). The paper does
  not print the E6/E8/E10 weights; they are obtained here by solving the
  isotropy conditions exactly: sum_alpha w_hat e_x^2 = 1 and every rank-2k
  moment tensor (k <= n) proportional to the fully symmetric delta product.

Isotropy of a weighted vector set (used both to solve and to check): the
rank-2k tensor T = sum w e...e is isotropic iff for every multi-index of
exponents (a_1..a_d) with sum 2k, sum w prod e_i^{a_i} equals
lambda * prod (a_i - 1)!! when all a_i are even, and 0 otherwise.
"""
from fractions import Fraction as Fr
from itertools import product

# --------------------------------------------------------------------------
# LB velocity sets (Sec. 3, Table 1; weights indexed by |c|^2)
# --------------------------------------------------------------------------

#: Table 1 rows, c_s^2 and w(|c|^2).  D3Q19 is the textbook cube lattice.
LATTICE_WEIGHTS = {
    "D2Q9": (2, Fr(1, 3), {0: Fr(4, 9), 1: Fr(1, 9), 2: Fr(1, 36)}),
    "D2Q13": (2, Fr(2, 5), {0: Fr(2, 5), 1: Fr(8, 75), 2: Fr(1, 25), 4: Fr(1, 300)}),
    "D2Q25": (2, Fr(4, 7), {0: Fr(72, 245), 1: Fr(16, 147), 2: Fr(16, 315),
                            4: Fr(1, 105), 5: Fr(8, 2205), 8: Fr(1, 8820)}),
    "D3Q19": (3, Fr(1, 3), {0: Fr(1, 3), 1: Fr(1, 18), 2: Fr(1, 36)}),
}


def shell(dim, n2):
    """All integer vectors of squared length n2 in `dim` dimensions."""
    m = int(n2 ** 0.5) + 1
    return [v for v in product(range(-m, m + 1), repeat=dim)
            if sum(x * x for x in v) == n2]


def lattice(name):
    """Return (dim, cs2, [(c, w)]) with the vectors ordered by |c|^2 then
    lexicographically.  D3Q19 excludes the |c|^2 = 3 corners."""
    dim, cs2, wmap = LATTICE_WEIGHTS[name]
    vel = []
    for n2 in sorted(wmap):
        for c in sorted(shell(dim, n2)):
            vel.append((c, wmap[n2]))
    return dim, cs2, vel


# --------------------------------------------------------------------------
# Isotropy algebra
# --------------------------------------------------------------------------

def dfact(n):
    """Double factorial (n)!! with (-1)!! = 1."""
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def exponents(dim, total):
    """All exponent tuples (a_1..a_dim) of non-negative ints summing to total."""
    if dim == 1:
        return [(total,)]
    out = []
    for a in range(total + 1):
        for rest in exponents(dim - 1, total - a):
            out.append((a,) + rest)
    return out


def moment(vecs, expo):
    """sum_v w_v prod_i v_i^{a_i} for a weighted vector list [(v, w)]."""
    s = Fr(0)
    for v, w in vecs:
        t = Fr(w)
        for vi, a in zip(v, expo):
            t *= Fr(vi) ** a
        s += t
    return s


def tensor_is_isotropic(vecs, dim, rank):
    """True iff the rank-`rank` moment tensor of vecs is lam * Delta^(rank)."""
    lam = None
    for expo in exponents(dim, rank):
        val = moment(vecs, expo)
        if any(a % 2 for a in expo):
            if val != 0:
                return False
            continue
        base = 1
        for a in expo:
            base *= dfact(a - 1)
        if lam is None:
            lam = val / base
        elif val != lam * base:
            return False
    return True


def isotropy_order(vecs, dim, max_rank=16):
    """Largest even rank 2n such that all tensors of rank 1..2n are isotropic
    (odd ranks must vanish).  Returns 2n."""
    order = 0
    for rank in range(1, max_rank + 1):
        if not tensor_is_isotropic(vecs, dim, rank):
            return order if rank % 2 == 0 else rank - 1
        if rank % 2 == 0:
            order = rank
    return order


# --------------------------------------------------------------------------
# Force stencils E_{2n}: weights by exact solve of the isotropy conditions
# --------------------------------------------------------------------------

#: Shells |e|^2 used by each stencil order (Sec. 2: E4 nearest neighbours,
#: E8 the 24-neighbour 2D stencil; E6, E10 and the 3D sets follow the same
#: rule: the fewest single-orbit shells that admit a solution).
FORCE_SHELLS = {
    (2, 4): (1, 2),
    (2, 6): (1, 2, 4),
    (2, 8): (1, 2, 4, 5, 8),
    (2, 10): (1, 2, 4, 5, 8, 9, 10),
    (3, 4): (1, 2),
    (3, 6): (1, 2, 3, 4),
    (3, 8): (1, 2, 3, 4, 5, 6, 8),
}


def solve_exact(a, b):
    """Gauss-Jordan elimination over Fractions for a square system a x = b."""
    n = len(a)
    m = [list(map(Fr, row)) + [Fr(bi)] for row, bi in zip(a, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        p = m[col][col]
        m[col] = [x / p for x in m[col]]
        for r in range(n):
            if r != col and m[r][col] != 0:
                f = m[r][col]
                m[r] = [x - f * y for x, y in zip(m[r], m[col])]
    return [m[r][n] for r in range(n)]


def _shell_moment(dim, n2, expo):
    return moment([(v, 1) for v in shell(dim, n2)], expo)


def force_weights(dim, order):
    """Exact w_hat(|e|^2) for the E_order stencil in `dim` dimensions.

    Conditions: sum w e_x^2 = 1, and for every even rank 2k with 4 <= 2k <= order
    the ratios between the even-exponent components of the rank-2k tensor
    equal those of Delta^(2k).  Odd components vanish by the cubic symmetry
    of complete shells; the mixed even ones are tied to the first one.
    """
    shells = FORCE_SHELLS[(dim, order)]
    rows, rhs = [], []
    rows.append([_shell_moment(dim, s, (2,) + (0,) * (dim - 1)) for s in shells])
    rhs.append(Fr(1))
    for rank in range(4, order + 1, 2):
        # canonical even-exponent components, sorted descending (cubic symmetry)
        comps = []
        for expo in exponents(dim, rank):
            if any(a % 2 for a in expo):
                continue
            key = tuple(sorted(expo, reverse=True))
            if key not in comps:
                comps.append(key)
        ref = comps[0]
        ref_iso = 1
        for a in ref:
            ref_iso *= dfact(a - 1)
        for comp in comps[1:]:
            iso = 1
            for a in comp:
                iso *= dfact(a - 1)
            # sum w [ m(comp) * ref_iso - m(ref) * iso ] = 0
            rows.append([_shell_moment(dim, s, comp) * ref_iso
                         - _shell_moment(dim, s, ref) * iso for s in shells])
            rhs.append(Fr(0))
    if len(rows) != len(shells):
        raise ValueError("stencil (%d, %d): %d conditions for %d shells"
                         % (dim, order, len(rows), len(shells)))
    sol = solve_exact(rows, rhs)
    return dict(zip(shells, sol))


def force_stencil(dim, order):
    """[(e, w_hat)] for every vector of the E_order stencil, ordered by shell
    then lexicographically."""
    w = force_weights(dim, order)
    out = []
    for n2 in sorted(w):
        for e in sorted(shell(dim, n2)):
            out.append((e, w[n2]))
    return out


def stencil_radius(dim, order):
    """Largest |e_i| component of the stencil (the psi halo width)."""
    return max(max(abs(x) for x in e) for e, _ in force_stencil(dim, order))


# --------------------------------------------------------------------------
# Taylor coefficients of the force operator (Sec. 2, Eq. (2))
# --------------------------------------------------------------------------

def taylor_coefficients(dim, order, kmax=None):
    """Coefficients a_k with sum_alpha w_hat e_i psi(x+e) = sum_k a_k
    d_i (lap)^k psi, valid while the rank-(2k+2) tensor is isotropic.

    For an isotropic rank-2m tensor sum w e^{2m} = lam_m Delta^(2m), the odd
    term of order 2m-1 in Eq. (2) contributes lam_m/(2m-1)! * (2m-1)!!/... ;
    concretely, contracting Delta^(2m) with e_i and 2m-1 gradients gives
    (2m-1)!! d_i lap^{m-1}, so a_{m-1} = lam_m (2m-1)!! / (2m-1)!.
    lam_m is read from the e_x^{2m} component: sum w e_x^{2m} = lam_m (2m-1)!!.
    """
    vecs = force_stencil(dim, order)
    kmax = order // 2 if kmax is None else kmax
    out = []
    for m in range(1, kmax + 1):
        exx = moment(vecs, (2 * m,) + (0,) * (dim - 1))
        lam = exx / dfact(2 * m - 1)
        fact = 1
        for j in range(2, 2 * m):
            fact *= j
        out.append(lam * dfact(2 * m - 1) / fact)
    return out


def mrt_gram_schmidt(name="D3Q19"):
    """Orthogonal (unweighted inner product) moment basis for a lattice, built
    by Gram-Schmidt from monomials ordered by degree.  Returns (rows, groups)
    where groups maps 'cons', 'bulk', 'shear', 'ghost' to row indices.

    Group reading: density and momentum are conserved; the trace c^2 carries
    bulk viscosity; the five traceless second-order moments carry shear
    viscosity (rate 1/tau); everything else is a non-hydrodynamic moment.
    """
    dim, cs2, vel = lattice(name)
    cs = [c for c, _ in vel]

    def vec(fn):
        return [Fr(fn(c)) for c in cs]

    if dim != 3:
        raise ValueError("MRT basis is built for 3D lattices only")
    cands = [
        ("cons", lambda c: 1),
        ("cons", lambda c: c[0]), ("cons", lambda c: c[1]), ("cons", lambda c: c[2]),
        ("bulk", lambda c: c[0] ** 2 + c[1] ** 2 + c[2] ** 2),
        ("shear", lambda c: 2 * c[0] ** 2 - c[1] ** 2 - c[2] ** 2),
        ("shear", lambda c: c[1] ** 2 - c[2] ** 2),
        ("shear", lambda c: c[0] * c[1]), ("shear", lambda c: c[1] * c[2]),
        ("shear", lambda c: c[0] * c[2]),
        ("ghost", lambda c: (c[0] ** 2 + c[1] ** 2 + c[2] ** 2) ** 2),
        ("ghost", lambda c: (c[0] ** 2 + c[1] ** 2 + c[2] ** 2) * c[0]),
        ("ghost", lambda c: (c[0] ** 2 + c[1] ** 2 + c[2] ** 2) * c[1]),
        ("ghost", lambda c: (c[0] ** 2 + c[1] ** 2 + c[2] ** 2) * c[2]),
        ("ghost", lambda c: (c[0] ** 2 + c[1] ** 2 + c[2] ** 2)
         * (2 * c[0] ** 2 - c[1] ** 2 - c[2] ** 2)),
        ("ghost", lambda c: (c[0] ** 2 + c[1] ** 2 + c[2] ** 2) * (c[1] ** 2 - c[2] ** 2)),
        ("ghost", lambda c: (c[1] ** 2 - c[2] ** 2) * c[0]),
        ("ghost", lambda c: (c[2] ** 2 - c[0] ** 2) * c[1]),
        ("ghost", lambda c: (c[0] ** 2 - c[1] ** 2) * c[2]),
    ]
    rows, groups = [], {"cons": [], "bulk": [], "shear": [], "ghost": []}
    for g, fn in cands:
        v = vec(fn)
        for r in rows:
            num = sum(a * b for a, b in zip(v, r))
            den = sum(b * b for b in r)
            v = [a - num / den * b for a, b in zip(v, r)]
        if all(x == 0 for x in v):
            raise ValueError("dependent moment in MRT basis")
        groups[g].append(len(rows))
        rows.append(v)
    return rows, groups
