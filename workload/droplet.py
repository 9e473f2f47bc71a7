"""Initial density fields of the droplet and flat-interface problems.

The droplet test (Sec. 3) places a disc of liquid in vapour on a periodic
grid with a tanh profile of width W.  The printed profile is garbled; the
reading used here is rho0 = (rl+rv)/2 - (rl-rv)/2 tanh(2 (r - R) / W) with r
the minimum-image distance to the centre (n/2 on nodes 0..n-1), so the grid
is symmetric under the square/cube group about the centre.

Jitter: i.i.d. U[-a, a] per node from splitmix64 (Steele, Lea & Flood 2014),
mapped to doubles by the top 53 bits.

Arrays are indexed [x, y] or [x, y, z].
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_uniform(seed, n, amp=1.0):
    """n doubles uniform in [-amp, amp) from the splitmix64 stream of `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (2.0 * u - 1.0) * amp


def _min_image(n):
    idx = np.arange(n, dtype=np.float64) - n // 2
    return (idx + n / 2.0) % n - n / 2.0


def droplet_rho(shape, radius, rho_l=2.0, rho_v=0.15, width=2.0, seed=None,
                jitter=1e-3, centre=None):
    """tanh droplet (disc in 2D, sphere in 3D) centred at n/2 per axis."""
    shape = tuple(int(s) for s in shape)
    grids = []
    for ax, n in enumerate(shape):
        if centre is None:
            d = _min_image(n)
        else:
            d = np.arange(n, dtype=np.float64) - centre[ax]
            d = (d + n / 2.0) % n - n / 2.0
        grids.append(d)
    mesh = np.meshgrid(*grids, indexing="ij")
    r = np.sqrt(sum(m * m for m in mesh))
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (r - radius) / width)
    if seed is not None and jitter:
        xi = splitmix64_uniform(seed, rho.size, jitter)
        # jitter stream in node order x fastest
        rho = rho + xi.reshape(shape[::-1]).transpose()
    return np.ascontiguousarray(rho)


def slab_rho(shape, thickness, rho_l=2.0, rho_v=0.15, width=2.0, axis=0):
    """Flat liquid slab of the given thickness centred on axis `axis`
    (the 1D flat-interface problem of Sec. 3)."""
    shape = tuple(int(s) for s in shape)
    n = shape[axis]
    d = np.abs(_min_image(n))
    prof = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (d - thickness / 2.0) / width)
    sl = [None] * len(shape)
    sl[axis] = slice(None)
    return np.ascontiguousarray(np.broadcast_to(prof[tuple(sl)], shape).astype(np.float64))


def sweep_items(n_items=64, seed=1906, side_range=(64, 512), sides=None):
    """Parameter draws of the droplet sweep: side ~ U{64..512},
    R ~ U{8..min(100, side//3)}, G ~ U[-5.5, -4.5], tau ~ U{0.8, 1.0, 1.2},
    order ~ U{4, 6, 8, 10}; jitter seed 1000 + i.  With `sides` fixed (e.g.
    256) every item uses that side."""
    rng = np.random.Generator(np.random.PCG64(seed))
    items = []
    for i in range(n_items):
        side = int(rng.integers(side_range[0], side_range[1] + 1)) if sides is None else int(sides)
        rmax = min(100, side // 3)
        R = int(rng.integers(8, rmax + 1))
        G = float(rng.uniform(-5.5, -4.5))
        tau = float(rng.choice([0.8, 1.0, 1.2]))
        order = int(rng.choice([4, 6, 8, 10]))
        items.append({"side": side, "R": R, "G": G, "tau": tau, "order": order,
                      "seed": 1000 + i})
    return items
