"""The allocation-free check (sc_lbm_check_noalloc) against sc_lbm_check,
through the C ABI: the same kernels on the same state, so every field of
the observables agrees bit for bit.  Two handles in a row, the second on a
smaller grid (fewer partial rows in the shared device array), then the
first again: the array keeps the last call's contents and each call must
still stand on its own."""
import pytest

from tests.gpu_helpers import say
from workload import droplet_rho

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1906_11027_amd import Sim  # noqa: E402
from paper_1906_11027_amd import sc_lbm as B  # noqa: E402


def _both(sim):
    rc_a, a = B.sc_lbm_check_noalloc(sim.h)
    rc_b, b = B.sc_lbm_check(sim.h)
    return (rc_a, a.as_dict()), (rc_b, b.as_dict())


def _same(x, y, label):
    (rc_a, a), (rc_b, b) = x, y
    say("%s: noalloc max|u| %.17g mass %.17g, check max|u| %.17g mass %.17g" % (
        label, a["max_u"], a["mass"], b["max_u"], b["mass"]))
    assert rc_a == rc_b == 0
    assert a == b, {k: (a[k], b[k]) for k in a if a[k] != b[k]}


def test_noalloc_check_matches_check_twice_then_smaller():
    big = Sim(droplet_rho((256, 256), 40, seed=2), "D2Q9", order=8)
    big.step(300)
    _same(*_both(big), "256^2 D2Q9 E8")
    small = Sim(droplet_rho((48, 40), 10, seed=3), "D2Q9", order=4, precision="fp64")
    small.step(50)
    _same(*_both(small), "48x40 D2Q9 E4 fp64")
    cube = Sim(droplet_rho((20, 18, 13), 5, seed=4), "D3Q19", order=8, collision="mrt")
    cube.step(20)
    _same(*_both(cube), "20x18x13 D3Q19 MRT E8")
    big.step(100)
    _same(*_both(big), "256^2 again")
    for s in (big, small, cube):
        s.close()


def test_noalloc_check_rejects_null():
    assert B.lib().sc_lbm_check_noalloc(None, None) == B.SC_E_INVAL
