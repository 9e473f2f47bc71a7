"""The product's Peng-Robinson set-up helper (paper_1906_11027_amd/eos.py)
against the oracle's independent EOS code and the paper's numbers (Sec. 3)."""
import warnings

import pytest

from oracle import eos as E
from paper_1906_11027_amd import eos as P

warnings.simplefilter("ignore")


def test_critical_point_matches_oracle_and_pr_constants():
    Tc, rc = P.critical_point()
    To, ro = E.critical_point()
    assert abs(Tc - To) < 1e-9 * To and abs(rc - ro) < 1e-6 * ro
    # Peng-Robinson: Tc = (Omega_b / Omega_a) a / (b R), Omega_a = 0.45724, Omega_b = 0.07780
    assert abs(Tc - 0.07780 * P.A / (0.45724 * P.B)) < 2e-4 * Tc


@pytest.mark.parametrize("Tr", [0.6, 0.725, 0.85, 0.95])
def test_maxwell_matches_oracle(Tr):
    a = P.maxwell(P.params_at(Tr))
    b = E.maxwell(E.eos_params(Tr))
    assert abs(a[0] - b[0]) < 1e-7 * b[0] and abs(a[1] - b[1]) < 1e-7 * b[1]


def test_density_ratio_range_of_the_sweep():
    """Sec. 3: 0.6 <= T/Tc <= 0.95 spans liquid/vapour density ratios of
    about 4 to 800 (read from the equal-area rule)."""
    lo = P.maxwell(P.params_at(0.95))
    hi = P.maxwell(P.params_at(0.6))
    assert 4.0 <= lo[1] / lo[0] < 6.0
    assert 700.0 < hi[1] / hi[0] < 1000.0


def test_params_at_alpha_is_one_at_tc():
    e = P.params_at(1.0)
    assert abs(e["alpha"] - 1.0) < 1e-15
    assert abs(e["T"] - P.critical_point()[0]) < 1e-15
