"""Host-side measurements of the experiments module on synthetic fields
(no GPU): contact angle of a circular cap, interface thickness of a tanh
profile."""
import math

import numpy as np
import pytest

from paper_1906_11027_amd import experiments as X


@pytest.mark.parametrize("theta", [40.0, 75.0, 90.0, 120.0, 150.0])
def test_contact_angle_of_a_circular_cap(theta):
    """A drop whose mid-density contour is a circle of radius R centred at
    height y_w - R cos(theta) meets the wall at theta."""
    shape, layers, R = (240, 140), 2, 45.0
    yw = layers - 0.5
    yc = yw - R * math.cos(math.radians(theta))
    x, y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    d = np.sqrt((x - 120.0) ** 2 + (y - yc) ** 2) - R
    rho = X.tanh_profile(d, 6.0, 0.5, 4.0)
    got, Rfit, hc = X.contact_angle(rho, layers, 6.0, 0.5)
    assert abs(got - theta) < 0.5, (got, theta)
    assert abs(Rfit - R) < 0.2


def test_contact_angle_limits():
    shape = (100, 60)
    film = np.full(shape, 6.0)
    assert X.contact_angle(film, 2, 6.0, 0.5)[0] == 0.0
    x, y = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    floating = X.tanh_profile(np.sqrt((x - 50.0) ** 2 + (y - 35.0) ** 2) - 10.0, 6.0, 0.5, 2.0)
    assert X.contact_angle(floating, 2, 6.0, 0.5)[0] == 180.0


@pytest.mark.parametrize("W,tol", [(20.0, 0.05), (5.0, 0.25)])
def test_interface_thickness_of_tanh(W, tol):
    """rho = m + a tanh(2 x / W) (vapour to liquid): the region
    1.05 rho_v .. 0.95 rho_l has a closed-form width; the crossings are
    placed by linear interpolation between nodes, which on a narrow profile
    errs by a fraction of a node in the curved tails."""
    rl, rv = 6.0, 0.5
    xs = np.arange(400) - 200.0
    prof = X.tanh_profile(-xs, rl, rv, W)   # liquid where -x < 0, i.e. on the right
    m, a = 0.5 * (rl + rv), 0.5 * (rl - rv)

    def x_of(level):   # solve m + a tanh(2 x / W) = level
        return 0.5 * W * math.atanh((level - m) / a)
    expect = abs(x_of(0.95 * rl) - x_of(1.05 * rv))
    got = X.interface_thickness(prof, rv, rl)
    assert abs(got - expect) < tol, (got, expect)
