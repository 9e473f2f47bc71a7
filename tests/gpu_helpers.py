"""Helpers for the GPU parity tests: map the library's stored state (post-
collision, shifted, library velocity order) to the oracle's pre-collision
distributions, and compare fields."""
import sys

import numpy as np

from paper_1906_11027_amd import sc_lbm as B


def lib_velocities(sim):
    return np.array(B.VELOCITIES[sim.p.lattice], dtype=np.int64)


# lattice weights by |c|^2 (Sec. 3, Table 1; D3Q19 the standard set)
_W = {"D2Q9": {0: 4 / 9, 1: 1 / 9, 2: 1 / 36},
      "D2Q13": {0: 2 / 5, 1: 8 / 75, 2: 1 / 25, 4: 1 / 300},
      "D2Q25": {0: 72 / 245, 1: 16 / 147, 2: 16 / 315, 4: 1 / 105, 5: 8 / 2205, 8: 1 / 8820},
      "D3Q19": {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}}


def lib_weights(lattice):
    """Weights in the library's velocity order."""
    vel = B.VELOCITIES[B.LATTICE[lattice]]
    return np.array([_W[lattice][sum(c * c for c in v)] for v in vel])


def pre_collision_from_state(sim, oracle_c):
    """f_b(x, t) = state_b(x - c_b) + w_b rho_ref, reordered to the oracle's
    velocity list `oracle_c` and indexed [q][x, y(, z)] in float64."""
    flat = sim.state().astype(np.float64)
    c = lib_velocities(sim)
    w = lib_weights(sim.lattice)
    shape = sim.shape
    out = np.zeros((len(c),) + shape)
    for b in range(len(c)):
        fb = flat[b * sim.n:(b + 1) * sim.n].reshape(shape[::-1]).transpose()
        fb = np.roll(fb, tuple(int(v) for v in c[b][:sim.dim]), axis=tuple(range(sim.dim)))
        out[b] = fb + w[b] * sim.rho_ref
    order = []
    for co in oracle_c:
        key = tuple(int(v) for v in co[:sim.dim])
        order.append([tuple(int(v) for v in cc) for cc in c].index(key))
    return out[order]


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def pre_collision_patch(state, sim, lo, size, oracle_c):
    """pre_collision_from_state restricted to the box [lo, lo + size) of the
    (periodic) grid, from a state array already copied to the host: f_b(x, t)
    = state_b(x - c_b) + w_b rho_ref in float64, oracle velocity order,
    indexed [q][x, y(, z)] over the box."""
    c = lib_velocities(sim)
    w = lib_weights(sim.lattice)
    shape, dim = sim.shape, sim.dim
    planes = state.reshape((len(c),) + tuple(shape[::-1]))    # [q][(z,) y, x]
    out = np.zeros((len(c),) + tuple(size))
    for b in range(len(c)):
        src = [(np.arange(lo[d], lo[d] + size[d]) - int(c[b][d])) % shape[d] for d in range(dim)]
        blk = planes[b][np.ix_(*src[::-1])]                    # [(z,) y, x] of the box
        out[b] = blk.transpose().astype(np.float64) + w[b] * sim.rho_ref
    order = []
    for co in oracle_c:
        key = tuple(int(v) for v in co[:dim])
        order.append([tuple(int(v) for v in cc[:dim]) for cc in c].index(key))
    return out[order]
