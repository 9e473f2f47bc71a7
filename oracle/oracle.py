"""Python handle on the FP64 CPU oracle (oracle/sc_oracle.c).

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the CPU-baseline
leg of bench.py may import this module; the GPU product path never does.

Observables follow the paper's spurious-velocity measures (Sec. 3, Fig. 3:
maximum and field-averaged |u|) and the pressure implied by the psi
definition of Sec. 3 (p = cs2 rho + G c0 psi^2 / 2 in lattice units).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "sc_oracle.c")

LATTICES = {"D2Q9": 0, "D3Q19": 1, "D2Q13": 2, "D2Q25": 3}
DIMS = {"D2Q9": 2, "D3Q19": 3, "D2Q13": 2, "D2Q25": 2}


def build(force=True):
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", SRC, "-o", LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("nz", ctypes.c_int), ("order", ctypes.c_int),
        ("G", ctypes.c_double), ("c0", ctypes.c_double),
        ("psi_kind", ctypes.c_int), ("psi0", ctypes.c_double),
        ("rho_psi", ctypes.c_double), ("tau", ctypes.c_double),
        ("collision", ctypes.c_int), ("s_bulk", ctypes.c_double),
        ("s_ghost", ctypes.c_double), ("forcing", ctypes.c_int),
        ("pr_a", ctypes.c_double), ("pr_b", ctypes.c_double), ("pr_R", ctypes.c_double),
        ("pr_T", ctypes.c_double), ("pr_alpha", ctypes.c_double),
        ("init", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(Params), dp]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.orc_get_f.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_f.argtypes = [ctypes.c_void_p, dp]
        L.orc_set_walls.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]
        L.orc_set_walls.restype = ctypes.c_int
        L.orc_force.argtypes = [ctypes.POINTER(Params), dp, dp]
        L.orc_force.restype = ctypes.c_int
        L.orc_lattice.argtypes = [ctypes.c_int, ip, ip, ip, dp, dp]
        L.orc_lattice.restype = ctypes.c_int
        L.orc_stencil.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp]
        L.orc_stencil.restype = ctypes.c_int
        L.orc_mrt_basis.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_mrt_basis.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads():
    """OpenMP threads the oracle's node loops use."""
    return lib().orc_num_threads()


def lattice_table(name):
    """(dim, c[Q,3] int, w[Q], cs2) as the oracle holds them."""
    c = np.zeros((25, 3), dtype=np.int32)
    w = np.zeros(25)
    dim, q = ctypes.c_int(), ctypes.c_int()
    cs2 = np.zeros(1)
    rc = lib().orc_lattice(LATTICES[name], ctypes.byref(dim), ctypes.byref(q),
                           c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w), _dp(cs2))
    assert rc == 0
    return dim.value, c[:q.value].copy(), w[:q.value].copy(), float(cs2[0])


def stencil_table(dim, order):
    """(e[n,3] int, w_hat[n]) of the E_order force stencil as the oracle holds it."""
    e = np.zeros((96, 3), dtype=np.int32)
    w = np.zeros(96)
    n = lib().orc_stencil(dim, order, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    if n <= 0:
        raise ValueError("no E%d stencil in %dD" % (order, dim))
    return e[:n].copy(), w[:n].copy()


def make_params(lattice="D2Q9", shape=(64, 64), order=4, G=-5.0, c0=1.0 / 3.0,
                psi="exp", psi0=1.0, rho_psi=1.0, tau=1.0, collision="srt",
                s_bulk=1.2, s_ghost=1.2, forcing="guo", eos=None, init="equilibrium"):
    """eos: for psi == "pr", a dict with a, b, R, T (absolute) and alpha.
    init: "equilibrium" (f = feq(rho0, 0)) or "rest" (f = feq(rho0, -F/(2 rho0)),
    zero forced velocity at t = 0)."""
    shape = tuple(shape)
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) > 2 else 1
    eos = eos or {}
    return Params(LATTICES[lattice], nx, ny, nz, order, G, c0,
                  {"exp": 0, "identity": 1, "pr": 2}[psi], psi0, rho_psi, tau,
                  {"srt": 0, "mrt": 1}[collision], s_bulk, s_ghost,
                  {"guo": 0, "edm": 1}[forcing], eos.get("a", 0.0), eos.get("b", 0.0),
                  eos.get("R", 0.0), eos.get("T", 0.0), eos.get("alpha", 0.0),
                  {"equilibrium": 0, "rest": 1}[init])


def force(psi_field, lattice="D2Q9", order=4, G=-5.0, c0=1.0 / 3.0):
    """Eq. (1) applied to an arbitrary psi field given as an array indexed
    [x, y] or [x, y, z].  Returns F with a leading component axis."""
    psi_field = np.asarray(psi_field, dtype=np.float64)
    shape = psi_field.shape
    p = make_params(lattice, shape, order, G, c0)
    flat = np.ascontiguousarray(psi_field.transpose()).ravel()  # x fastest
    dim = len(shape)
    F = np.zeros(dim * flat.size)
    assert lib().orc_force(ctypes.byref(p), _dp(flat), _dp(F)) == 0
    F = F.reshape((dim,) + shape[::-1])
    return np.stack([F[d].transpose() for d in range(dim)])


class Oracle:
    """FP64 reference simulation.  Fields are returned indexed [x, y(, z)]."""

    def __init__(self, rho0, lattice="D2Q9", order=4, G=-5.0, c0=1.0 / 3.0,
                 psi="exp", psi0=1.0, rho_psi=1.0, tau=1.0, collision="srt",
                 s_bulk=1.2, s_ghost=1.2, forcing="guo", eos=None, init="equilibrium"):
        rho0 = np.asarray(rho0, dtype=np.float64)
        self.shape = rho0.shape
        self.dim = DIMS[lattice]
        assert rho0.ndim == self.dim
        self.lattice, self.order, self.G, self.c0 = lattice, order, G, c0
        self.psi_kind, self.psi0, self.rho_psi = psi, psi0, rho_psi
        self.tau = tau
        self.p = make_params(lattice, self.shape, order, G, c0, psi, psi0, rho_psi,
                             tau, collision, s_bulk, s_ghost, forcing, eos, init)
        self.eos = eos
        self.n = rho0.size
        self._dim, self.c, self.w, self.cs2 = lattice_table(lattice)
        self.q = len(self.w)
        flat = np.ascontiguousarray(rho0.transpose()).ravel()
        self.h = lib().orc_create(ctypes.byref(self.p), _dp(flat))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.steps = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def _unflat(self, a):
        return a.reshape(self.shape[::-1]).transpose()

    def step(self, n=1):
        lib().orc_step(self.h, n)
        self.steps += n
        return self

    def fields(self):
        n, d = self.n, self.dim
        rho, psi = np.zeros(n), np.zeros(n)
        F, u = np.zeros(d * n), np.zeros(d * n)
        lib().orc_fields(self.h, _dp(rho), _dp(psi), _dp(F), _dp(u))
        return {
            "rho": self._unflat(rho), "psi": self._unflat(psi),
            "F": np.stack([self._unflat(F[k * n:(k + 1) * n]) for k in range(d)]),
            "u": np.stack([self._unflat(u[k * n:(k + 1) * n]) for k in range(d)]),
        }

    def get_f(self):
        """Distributions f[q] indexed like the fields (pre-collision, time t)."""
        f = np.zeros(self.q * self.n)
        lib().orc_get_f(self.h, _dp(f))
        return np.stack([self._unflat(f[b * self.n:(b + 1) * self.n]) for b in range(self.q)])

    def set_f(self, f):
        flat = np.concatenate([np.ascontiguousarray(np.asarray(fb, dtype=np.float64)
                                                    .transpose()).ravel() for fb in f])
        lib().orc_set_f(self.h, _dp(flat))

    def mrt_basis(self):
        M, nn, S = np.zeros(19 * 19), np.zeros(19), np.zeros(19)
        if lib().orc_mrt_basis(self.h, _dp(M), _dp(nn), _dp(S)) != 0:
            raise ValueError("not an MRT simulation")
        return M.reshape(19, 19), nn, S

    def set_walls(self, solid, rho_w):
        """Solid mask indexed like the fields (nonzero = solid) and virtual
        wall density (the populations are kept).  None removes the walls."""
        if solid is None:
            self.solid = None
            assert lib().orc_set_walls(self.h, None, 0.0) == 0
            return self
        m = np.ascontiguousarray(np.asarray(solid).transpose()).ravel().astype(np.uint8)
        assert m.size == self.n
        assert lib().orc_set_walls(self.h, m.ctypes.data_as(ctypes.c_void_p), float(rho_w)) == 0
        self.solid = np.asarray(solid).astype(bool)
        return self

    def observables(self):
        return observables(self.fields(), self.cs2, self.G, self.c0, getattr(self, "solid", None))


def observables(fl, cs2, G, c0, solid=None):
    """(The pressure uses the psi definition of Sec. 3 for every psi kind:
    p = cs2 rho + G c0 psi^2 / 2, which equals the EOS pressure for "pr".)
    With walls, the velocity norms run over the fluid nodes; the mass
    counts every population (solid nodes hold those in transit)."""
    return _observables(fl, cs2, G, c0, solid)


def _observables(fl, cs2, G, c0, solid=None):
    """Reductions every K steps: mass, momentum, spurious-velocity norms
    (maximum and field average, Sec. 3 Fig. 3), Laplace pressure jump
    between the centre node and the corner node, equivalent radius."""
    rho, psi, u = fl["rho"], fl["psi"], fl["u"]
    dim = rho.ndim
    umag = np.sqrt((u ** 2).sum(axis=0))
    rho_fluid = rho
    if solid is not None:
        umag = umag[~solid]
        rho_fluid = rho[~solid]
    p = cs2 * rho + 0.5 * G * c0 * psi ** 2
    centre = tuple(s // 2 for s in rho.shape)
    corner = (0,) * dim
    rin, rout = rho[centre], rho[corner]
    vol = (rho - rout).sum() / (rin - rout) if rin != rout else 0.0
    if dim == 2:
        radius = np.sqrt(max(vol, 0.0) / np.pi)
    else:
        radius = (3.0 * max(vol, 0.0) / (4.0 * np.pi)) ** (1.0 / 3.0)
    return {
        "mass": rho.sum(),
        "mom": (rho[None] * u).reshape(dim, -1).sum(axis=1),
        "max_u": umag.max(), "mean_u": umag.mean(),
        "l2_u": np.sqrt((umag ** 2).mean()),
        "rho_in": rin, "rho_out": rout,
        "p_in": p[centre], "p_out": p[corner], "dp": p[centre] - p[corner],
        "radius": radius,
        "rho_min": rho_fluid.min(), "rho_max": rho_fluid.max(),
    }
