"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/sc_lbm.h declares, and rejects invalid parameter sets before any
device call.  No kernel is launched here."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_1906_11027_amd import sc_lbm as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sc_lbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_(?:lbm|nn)_[a-z0-9_]+)\s*\(", src)))


def test_header_lists_match_binding():
    assert declared_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def _c_layout(tmp_path, struct, fields):
    """sizeof and field offsets as the C compiler lays the header out."""
    prog = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sc_lbm.h"', 'int main(void){',
             'printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines.append('return 0;}')
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    return [int(v) for v in subprocess.check_output([str(exe)]).split()]


@pytest.mark.parametrize("cls,name", [(B.sc_lbm_params, "sc_lbm_params"), (B.sc_lbm_obs, "sc_lbm_obs")])
def test_struct_layout_matches_header(tmp_path, cls, name):
    fields = [f for f, _ in cls._fields_]
    got = _c_layout(tmp_path, name, fields)
    assert got[0] == ctypes.sizeof(cls)
    assert got[1:] == [getattr(cls, f).offset for f in fields]


def test_defaults():
    p = B.sc_lbm_default_params()
    assert (p.lattice, p.nx, p.ny, p.nz, p.order) == (0, 64, 64, 1, 4)
    assert p.G == -5.0 and abs(p.c0 - 1 / 3) < 1e-16 and p.tau == 1.0
    assert p.variant == -1 and p.obs_every == 100
    assert p.init == B.SC_INIT_EQUILIBRIUM and p.forcing == B.SC_GUO
    assert p.rho_ref == B.SC_RHO_REF_AUTO
    assert B.sc_lbm_state_bytes(p) == 9 * 64 * 64 * 4
    p.precision = B.SC_FP64
    assert B.sc_lbm_state_bytes(p) == 9 * 64 * 64 * 8


@pytest.mark.parametrize("field,value,code", [
    ("lattice", 7, B.SC_E_INVAL),
    ("nx", 0, B.SC_E_INVAL),
    ("nz", 2, B.SC_E_INVAL),          # 2D lattice with nz > 1
    ("order", 5, B.SC_E_INVAL),
    ("tau", 0.5, B.SC_E_INVAL),
    ("tau", float("nan"), B.SC_E_INVAL),
    ("psi_kind", 3, B.SC_E_INVAL),
    ("collision", B.SC_MRT, B.SC_E_UNSUPPORTED),   # MRT is D3Q19 only
    ("precision", 9, B.SC_E_INVAL),
    ("variant", 99, B.SC_E_INVAL),
    ("G", float("inf"), B.SC_E_INVAL),
    ("init", 2, B.SC_E_INVAL),
    ("rho_ref", float("inf"), B.SC_E_INVAL),
    ("rho_ref", float("nan"), B.SC_E_INVAL),
])
def test_invalid_parameters_rejected(field, value, code):
    p = B.sc_lbm_default_params()
    setattr(p, field, value)
    assert B.sc_lbm_state_bytes(p) == 0
    h = ctypes.c_void_p()
    assert B.lib().sc_lbm_create(ctypes.byref(p), None, None, None, None, ctypes.byref(h)) == code
    assert h.value is None


def test_shift_accessors_on_null_handles():
    L = B.lib()
    assert math.isnan(L.sc_lbm_rho_ref(None)) and math.isnan(L.sc_lbm_batch_rho_ref(None))


def test_batch_items_must_share_the_shift():
    # checked before any device call
    a = B.make_params("D2Q9", (16, 16))
    b = B.make_params("D2Q9", (16, 16), rho_ref=1.0)
    with pytest.raises(B.ScError) as ei:
        B.sc_lbm_batch_create([a, b])
    assert ei.value.code == B.SC_E_INVAL


def test_make_params_shift():
    assert B.make_params().rho_ref == B.SC_RHO_REF_AUTO
    assert B.make_params(rho_ref=0.25).rho_ref == 0.25
    # any negative shift asks for the automatic one and is a valid problem
    p = B.make_params(rho_ref=-3.0)
    assert B.sc_lbm_state_bytes(p) == 9 * 64 * 64 * 4


def test_largest_velocity_plane():
    # one velocity plane must stay below 4 GiB (32-bit byte offsets)
    p = B.sc_lbm_default_params()
    p.nx, p.ny = 65536, 16383
    assert B.sc_lbm_state_bytes(p) == 9 * 65536 * 16383 * 4
    p.ny = 16384
    assert B.sc_lbm_state_bytes(p) == 0
    h = ctypes.c_void_p()
    assert B.lib().sc_lbm_create(ctypes.byref(p), None, None, None, None, ctypes.byref(h)) == B.SC_E_UNSUPPORTED
    p.precision, p.ny = B.SC_FP64, 8191
    assert B.sc_lbm_state_bytes(p) == 9 * 65536 * 8191 * 8
    p.ny = 8192
    assert B.sc_lbm_state_bytes(p) == 0


def test_3d_order_10_unsupported():
    p = B.sc_lbm_default_params()
    p.lattice, p.nz, p.order = B.SC_D3Q19, 8, 10
    h = ctypes.c_void_p()
    assert B.lib().sc_lbm_create(ctypes.byref(p), None, None, None, None, ctypes.byref(h)) == B.SC_E_UNSUPPORTED


def test_single_buffer_rejected():
    p = B.sc_lbm_default_params()
    h = ctypes.c_void_p()
    assert B.lib().sc_lbm_create(ctypes.byref(p), None, ctypes.c_void_p(1234), None, None,
                                 ctypes.byref(h)) == B.SC_E_INVAL


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert B.sc_lbm_strerror(code)
    n9 = B.sc_lbm_num_variants(B.make_params("D2Q9"))
    n19 = B.sc_lbm_num_variants(B.make_params("D3Q19", (8, 8, 8)))
    nw = B.sc_lbm_num_variants(B.make_params("D2Q25"))
    assert n9 >= 1 and n19 >= 1 and nw >= 1
    # D2Q9 with the exact difference method runs in the any-lattice family
    assert B.sc_lbm_num_variants(B.make_params("D2Q9", forcing="edm")) == nw
    assert B.sc_lbm_num_variants(B.make_params("D2Q9", order=5)) == 0


def test_batch_autotune_rejects_before_any_device_call():
    L = B.lib()
    v, ms = ctypes.c_int32(), ctypes.c_double()
    assert L.sc_lbm_batch_autotune(None, 1, 32, ctypes.byref(v), ctypes.byref(ms)) == B.SC_E_INVAL
    arr = (B.sc_lbm_params * 1)(B.make_params("D2Q9", (16, 16)))
    assert L.sc_lbm_batch_autotune(arr, 0, 32, ctypes.byref(v), ctypes.byref(ms)) == B.SC_E_INVAL
    assert L.sc_lbm_batch_autotune(arr, 1, 0, ctypes.byref(v), ctypes.byref(ms)) == B.SC_E_INVAL


def test_conv_shapes_rejected_before_any_device_call():
    """The MFMA convolution kernels address one image's channels with
    32-bit element offsets: images whose 32 channels exceed 2^31 elements,
    and unsupported channel counts, are rejected on the host."""
    L = B.lib()
    p = ctypes.c_void_p(4096)   # never dereferenced: every call below is rejected first
    # 8192 x 8192 x 32 = 2^31 elements
    assert L.sc_nn_conv3x3_fwd(p, p, p, p, 1, 32, 32, 8192, 8192, None) == B.SC_E_INVAL
    assert L.sc_nn_conv3x3_fwd(p, p, p, p, 1, 33, 32, 16, 16, None) == B.SC_E_INVAL
    assert L.sc_nn_conv3x3_fwd(p, p, p, p, 1, 32, 16, 16, 16, None) == B.SC_E_INVAL
    assert L.sc_nn_conv3x3_fwd(p, p, p, p, 0, 32, 32, 16, 16, None) == B.SC_E_INVAL
    assert L.sc_nn_conv3x3_bwd_weight(p, p, p, 4, p, p, 1, 32, 32, 8192, 8192, None) == B.SC_E_INVAL
