"""ctypes binding of libsc_lbm.so (include/sc_lbm.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module only
converts numpy arrays and torch device buffers/streams to plain pointers.
There is no CPU fallback: if the shared library is missing, importing the
binding raises.

Field arrays returned by :class:`Sim` are indexed [x, y] or [x, y, z]
(vector fields with a leading component axis); the C ABI itself uses flat
node order i = x + nx (y + ny z).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsc_lbm.so")

SC_OK, SC_E_INVAL, SC_E_NOMEM, SC_E_DEVICE, SC_E_UNSUPPORTED, SC_E_NONFINITE = 0, -1, -2, -3, -4, -5
SC_D2Q9, SC_D3Q19, SC_D2Q13, SC_D2Q25 = 0, 1, 2, 3
SC_PSI_EXP, SC_PSI_IDENTITY, SC_PSI_PR = 0, 1, 2
SC_GUO, SC_EDM = 0, 1
SC_SRT, SC_MRT = 0, 1
SC_FP32_SHIFTED, SC_FP64 = 0, 1
SC_INIT_EQUILIBRIUM, SC_INIT_REST = 0, 1
SC_RHO_REF_AUTO = -1.0

LATTICE = {"D2Q9": SC_D2Q9, "D3Q19": SC_D3Q19, "D2Q13": SC_D2Q13, "D2Q25": SC_D2Q25}
Q = {SC_D2Q9: 9, SC_D3Q19: 19, SC_D2Q13: 13, SC_D2Q25: 25}


class sc_lbm_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("order", ctypes.c_int32), ("psi_kind", ctypes.c_int32),
        ("G", ctypes.c_double), ("c0", ctypes.c_double), ("psi0", ctypes.c_double),
        ("rho_psi", ctypes.c_double), ("tau", ctypes.c_double),
        ("collision", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("s_bulk", ctypes.c_double), ("s_ghost", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("obs_every", ctypes.c_int32), ("variant", ctypes.c_int32), ("forcing", ctypes.c_int32),
        ("init", ctypes.c_int32),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double), ("eos_R", ctypes.c_double),
        ("eos_T", ctypes.c_double), ("eos_alpha", ctypes.c_double),
    ]


class sc_lbm_obs(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double), ("mom", ctypes.c_double * 3),
        ("max_u", ctypes.c_double), ("mean_u", ctypes.c_double), ("l2_u", ctypes.c_double),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("p_in", ctypes.c_double), ("p_out", ctypes.c_double), ("dp", ctypes.c_double),
        ("radius", ctypes.c_double), ("rho_min", ctypes.c_double), ("rho_max", ctypes.c_double),
        ("d_max_u", ctypes.c_double),
        ("nonfinite", ctypes.c_int64), ("converged_by", ctypes.c_int32), ("status", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["mom"] = list(self.mom)
        return d


#: every symbol include/sc_lbm.h declares
EXPORTS = [
    "sc_lbm_default_params", "sc_lbm_state_bytes", "sc_lbm_create", "sc_lbm_step",
    "sc_lbm_force", "sc_lbm_observe", "sc_lbm_check", "sc_lbm_check_noalloc", "sc_lbm_set_state", "sc_lbm_state_ptr",
    "sc_lbm_variant_name", "sc_lbm_num_variants", "sc_lbm_destroy", "sc_lbm_strerror", "sc_lbm_set_walls",
    "sc_lbm_steps_per_launch",
    "sc_lbm_last_error_detail", "sc_lbm_stream", "sc_lbm_rho_ref",
    "sc_lbm_batch_create", "sc_lbm_batch_step", "sc_lbm_batch_observe", "sc_lbm_batch_status",
    "sc_lbm_batch_active", "sc_lbm_batch_rho_ref", "sc_lbm_batch_variant_name", "sc_lbm_batch_num_variants", "sc_lbm_batch_promote", "sc_lbm_batch_autotune", "sc_lbm_batch_destroy", "sc_lbm_autotune",
    "sc_nn_conv3x3_fwd", "sc_nn_conv3x3_fwd_tanh", "sc_nn_conv3x3_bwd_data", "sc_nn_conv3x3_bwd_data_tanh",
    "sc_nn_bwd_weight_scratch_floats",
    "sc_nn_conv3x3_bwd_weight", "sc_nn_tanh_fwd", "sc_nn_tanh_bwd", "sc_nn_mse", "sc_nn_adam",
    "sc_nn_to_bf16", "sc_nn_features", "sc_nn_start_field",
]

#: velocity order of the state buffers (include/sc_lbm.h)
VELOCITIES = {
    SC_D2Q9: [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
    SC_D3Q19: [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
               (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
               (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)],
    SC_D2Q13: [(0, 0), (-1, 0), (0, -1), (0, 1), (1, 0), (-1, -1), (-1, 1), (1, -1), (1, 1),
               (-2, 0), (0, -2), (0, 2), (2, 0)],
}
VELOCITIES[SC_D2Q25] = VELOCITIES[SC_D2Q13] + [(-2, -1), (-2, 1), (-1, -2), (-1, 2), (1, -2), (1, 2), (2, -1),
                                               (2, 1), (-2, -2), (-2, 2), (2, -2), (2, 2)]

_lib = None


def lib():
    """Load libsc_lbm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsc_lbm.so is not built (run __graft_entry__.build()); "
                           "there is no CPU fallback")
    # torch ships its own libamdhip64 (same soname, loaded by file name).  Load
    # it first so this library binds to that copy: two HIP runtimes in one
    # process do not share the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, dp = ctypes.c_void_p, P(ctypes.c_double)
    L.sc_lbm_default_params.argtypes = [P(sc_lbm_params)]
    L.sc_lbm_default_params.restype = None
    L.sc_lbm_state_bytes.argtypes = [P(sc_lbm_params)]
    L.sc_lbm_state_bytes.restype = ctypes.c_size_t
    L.sc_lbm_create.argtypes = [P(sc_lbm_params), dp, vp, vp, vp, P(vp)]
    L.sc_lbm_create.restype = ctypes.c_int
    L.sc_lbm_step.argtypes = [vp, ctypes.c_int64, ctypes.c_double, P(ctypes.c_int64)]
    L.sc_lbm_step.restype = ctypes.c_int
    L.sc_lbm_force.argtypes = [vp, dp, dp]
    L.sc_lbm_force.restype = ctypes.c_int
    L.sc_lbm_observe.argtypes = [vp, P(sc_lbm_obs), dp, dp, vp]
    L.sc_lbm_observe.restype = ctypes.c_int
    L.sc_lbm_check.argtypes = [vp, P(sc_lbm_obs)]
    L.sc_lbm_check.restype = ctypes.c_int
    L.sc_lbm_check_noalloc.argtypes = [vp, P(sc_lbm_obs)]
    L.sc_lbm_check_noalloc.restype = ctypes.c_int
    L.sc_lbm_set_state.argtypes = [vp, vp, ctypes.c_int64]
    L.sc_lbm_set_state.restype = ctypes.c_int
    L.sc_lbm_state_ptr.argtypes = [vp]
    L.sc_lbm_state_ptr.restype = vp
    L.sc_lbm_variant_name.argtypes = [vp]
    L.sc_lbm_variant_name.restype = ctypes.c_char_p
    L.sc_lbm_num_variants.argtypes = [P(sc_lbm_params)]
    L.sc_lbm_steps_per_launch.argtypes = [vp]
    L.sc_lbm_steps_per_launch.restype = ctypes.c_int
    L.sc_lbm_set_walls.argtypes = [vp, vp, ctypes.c_double]
    L.sc_lbm_set_walls.restype = ctypes.c_int
    L.sc_lbm_num_variants.restype = ctypes.c_int
    L.sc_lbm_destroy.argtypes = [vp]
    L.sc_lbm_destroy.restype = None
    L.sc_lbm_strerror.argtypes = [ctypes.c_int]
    L.sc_lbm_strerror.restype = ctypes.c_char_p
    L.sc_lbm_batch_create.argtypes = [P(sc_lbm_params), ctypes.c_int32, P(dp), vp, P(vp)]
    L.sc_lbm_batch_create.restype = ctypes.c_int
    L.sc_lbm_batch_step.argtypes = [vp, ctypes.c_int64, ctypes.c_double, P(ctypes.c_int64)]
    L.sc_lbm_batch_step.restype = ctypes.c_int
    L.sc_lbm_batch_observe.argtypes = [vp, ctypes.c_int32, P(sc_lbm_obs), dp, dp]
    L.sc_lbm_batch_observe.restype = ctypes.c_int
    L.sc_lbm_batch_status.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_int32)]
    L.sc_lbm_batch_status.restype = ctypes.c_int
    L.sc_lbm_batch_active.argtypes = [vp]
    L.sc_lbm_batch_active.restype = ctypes.c_int32
    L.sc_lbm_batch_destroy.argtypes = [vp]
    L.sc_lbm_batch_destroy.restype = None
    L.sc_lbm_autotune.argtypes = [P(sc_lbm_params), ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_double)]
    L.sc_lbm_autotune.restype = ctypes.c_int
    i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.sc_nn_conv3x3_fwd.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, i32, vp]
    L.sc_nn_conv3x3_fwd_tanh.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, i32, vp]
    L.sc_nn_conv3x3_bwd_data_tanh.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, vp]
    L.sc_nn_conv3x3_bwd_data.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, i32, vp]
    L.sc_nn_bwd_weight_scratch_floats.argtypes = [i32, i32, i32]
    L.sc_nn_bwd_weight_scratch_floats.restype = i32
    L.sc_nn_conv3x3_bwd_weight.argtypes = [vp, vp, vp, i32, vp, vp, i32, i32, i32, i32, i32, vp]
    L.sc_nn_tanh_fwd.argtypes = [vp, i64, vp]
    L.sc_nn_tanh_bwd.argtypes = [vp, vp, i64, vp]
    L.sc_nn_mse.argtypes = [vp, vp, vp, vp, i32, i64, vp]
    L.sc_nn_adam.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
    L.sc_nn_to_bf16.argtypes = [vp, vp, i64, vp]
    L.sc_nn_features.argtypes = [vp, vp, i32, i32, i32, f32, vp]
    L.sc_nn_start_field.argtypes = [vp, vp, vp, vp, i32, i32, i32, f32, ctypes.c_double, ctypes.c_double, vp]
    for name in ("sc_nn_conv3x3_fwd", "sc_nn_conv3x3_fwd_tanh", "sc_nn_conv3x3_bwd_data",
                 "sc_nn_conv3x3_bwd_data_tanh", "sc_nn_conv3x3_bwd_weight", "sc_nn_tanh_fwd",
                 "sc_nn_tanh_bwd", "sc_nn_mse", "sc_nn_adam", "sc_nn_to_bf16", "sc_nn_features",
                 "sc_nn_start_field"):
        getattr(L, name).restype = ctypes.c_int
    L.sc_lbm_stream.argtypes = [vp]
    L.sc_lbm_stream.restype = vp
    L.sc_lbm_rho_ref.argtypes = [vp]
    L.sc_lbm_rho_ref.restype = ctypes.c_double
    L.sc_lbm_batch_rho_ref.argtypes = [vp]
    L.sc_lbm_batch_rho_ref.restype = ctypes.c_double
    L.sc_lbm_batch_variant_name.argtypes = [vp]
    L.sc_lbm_batch_promote.argtypes = [vp]
    L.sc_lbm_batch_num_variants.argtypes = []
    L.sc_lbm_batch_num_variants.restype = ctypes.c_int32
    L.sc_lbm_batch_promote.restype = ctypes.c_int
    L.sc_lbm_batch_autotune.argtypes = [ctypes.POINTER(sc_lbm_params), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    L.sc_lbm_batch_autotune.restype = ctypes.c_int
    L.sc_lbm_batch_variant_name.restype = ctypes.c_char_p
    L.sc_lbm_last_error_detail.argtypes = []
    L.sc_lbm_last_error_detail.restype = ctypes.c_char_p
    _lib = L
    return L


class ScError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().sc_lbm_strerror(code).decode()
        detail = lib().sc_lbm_last_error_detail().decode()
        super().__init__("%s failed: %s (%d)%s" % (what, msg, code, (" [" + detail + "]") if detail else ""))


def _check(code, what):
    if code != SC_OK:
        raise ScError(code, what)
    return code


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def sc_lbm_default_params():
    p = sc_lbm_params()
    lib().sc_lbm_default_params(ctypes.byref(p))
    return p


def sc_lbm_state_bytes(p):
    return lib().sc_lbm_state_bytes(ctypes.byref(p))


def sc_lbm_create(p, rho_init=None, dev_a=None, dev_b=None, stream=None):
    """Returns the handle (int).  rho_init: flat float64 [N] in node order."""
    h = ctypes.c_void_p()
    if rho_init is not None:
        rho_init = np.ascontiguousarray(rho_init, dtype=np.float64)
    rc = lib().sc_lbm_create(ctypes.byref(p), _dptr(rho_init), dev_a, dev_b, stream, ctypes.byref(h))
    _check(rc, "sc_lbm_create")
    return h.value


def sc_lbm_step(h, max_steps, tol=0.0):
    done = ctypes.c_int64(0)
    rc = lib().sc_lbm_step(h, int(max_steps), float(tol), ctypes.byref(done))
    return rc, done.value


def sc_lbm_force(h, n, dim, psi_in=None):
    F = np.zeros(dim * n)
    if psi_in is not None:
        psi_in = np.ascontiguousarray(psi_in, dtype=np.float64)
    _check(lib().sc_lbm_force(h, _dptr(psi_in), _dptr(F)), "sc_lbm_force")
    return F


def sc_lbm_observe(h, rho_out=None, u_out=None, f_out=None):
    o = sc_lbm_obs()
    fptr = None if f_out is None else f_out.ctypes.data_as(ctypes.c_void_p)
    rc = lib().sc_lbm_observe(h, ctypes.byref(o), _dptr(rho_out), _dptr(u_out), fptr)
    if rc not in (SC_OK, SC_E_NONFINITE):
        raise ScError(rc, "sc_lbm_observe")
    return rc, o


def sc_lbm_check(h):
    o = sc_lbm_obs()
    rc = lib().sc_lbm_check(h, ctypes.byref(o))
    if rc not in (SC_OK, SC_E_NONFINITE):
        raise ScError(rc, "sc_lbm_check")
    return rc, o


def sc_lbm_check_noalloc(h):
    o = sc_lbm_obs()
    rc = lib().sc_lbm_check_noalloc(h, ctypes.byref(o))
    if rc not in (SC_OK, SC_E_NONFINITE):
        raise ScError(rc, "sc_lbm_check_noalloc")
    return rc, o


def sc_lbm_set_state(h, f_in, step):
    _check(lib().sc_lbm_set_state(h, f_in.ctypes.data_as(ctypes.c_void_p), int(step)), "sc_lbm_set_state")


def sc_lbm_set_walls(h, solid, rho_w):
    """solid: flat uint8 [N] in node order, or None to remove the walls."""
    ptr = None
    if solid is not None:
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        ptr = solid.ctypes.data_as(ctypes.c_void_p)
    _check(lib().sc_lbm_set_walls(h, ptr, float(rho_w)), "sc_lbm_set_walls")


def sc_lbm_state_ptr(h):
    return lib().sc_lbm_state_ptr(h)


def sc_lbm_autotune(p, steps=20):
    """Returns (best variant, ms per step) and records the choice."""
    v, ms = ctypes.c_int32(), ctypes.c_double()
    _check(lib().sc_lbm_autotune(ctypes.byref(p), int(steps), ctypes.byref(v), ctypes.byref(ms)), "sc_lbm_autotune")
    return v.value, ms.value


def sc_lbm_variant_name(h):
    return lib().sc_lbm_variant_name(h).decode()


def sc_lbm_num_variants(p):
    """Launch shapes of the kernel family serving parameter set p."""
    return lib().sc_lbm_num_variants(ctypes.byref(p))


def sc_lbm_destroy(h):
    lib().sc_lbm_destroy(h)


def sc_lbm_strerror(code):
    return lib().sc_lbm_strerror(code).decode()


# ---------------------------------------------------------------------------
# convenience handle
# ---------------------------------------------------------------------------

def make_params(lattice="D2Q9", shape=(64, 64), order=4, G=-5.0, c0=1.0 / 3.0, psi="exp",
                psi0=1.0, rho_psi=1.0, tau=1.0, collision="srt", precision="fp32",
                s_bulk=1.2, s_ghost=1.2, rho_ref="auto", obs_every=100, variant=-1, forcing="guo", eos=None,
                init="equilibrium"):
    """eos: for psi == "pr", a dict with a, b, R, T (absolute) and alpha.
    init: "equilibrium" (f = feq(rho0, 0)) or "rest" (f = feq(rho0, -F/(2 rho0)):
    the forced velocity is zero at t = 0).
    rho_ref: the storage shift, or "auto" (the median initial density)."""
    p = sc_lbm_default_params()
    p.lattice = LATTICE[lattice]
    shape = tuple(int(s) for s in shape)
    p.nx, p.ny = shape[0], shape[1]
    p.nz = shape[2] if len(shape) > 2 else 1
    p.order = order
    p.psi_kind = {"exp": SC_PSI_EXP, "identity": SC_PSI_IDENTITY, "pr": SC_PSI_PR}[psi]
    p.forcing = {"guo": SC_GUO, "edm": SC_EDM}[forcing]
    if eos:
        p.eos_a, p.eos_b, p.eos_R, p.eos_T, p.eos_alpha = eos["a"], eos["b"], eos["R"], eos["T"], eos["alpha"]
    p.G, p.c0, p.psi0, p.rho_psi, p.tau = G, c0, psi0, rho_psi, tau
    p.collision = {"srt": SC_SRT, "mrt": SC_MRT}[collision]
    p.precision = {"fp32": SC_FP32_SHIFTED, "fp64": SC_FP64}[precision]
    p.s_bulk, p.s_ghost = s_bulk, s_ghost
    p.rho_ref = SC_RHO_REF_AUTO if isinstance(rho_ref, str) and rho_ref == "auto" else float(rho_ref)
    p.obs_every, p.variant = obs_every, variant
    p.init = {"equilibrium": SC_INIT_EQUILIBRIUM, "rest": SC_INIT_REST}[init]
    return p


class Sim:
    """One periodic domain on the GPU.  Device memory and the stream come
    from torch when `use_torch` is set (the default when torch sees a GPU)."""

    def __init__(self, rho0, lattice="D2Q9", use_torch=None, stream=None, **kw):
        rho0 = np.asarray(rho0, dtype=np.float64)
        self.shape = rho0.shape
        self.dim = rho0.ndim
        self.p = make_params(lattice, self.shape, **kw)
        self.q = Q[self.p.lattice]
        self.n = int(rho0.size)
        self.lattice = lattice
        self._bufs = None
        dev_a = dev_b = None
        if use_torch is None:
            try:
                import torch
                use_torch = torch.cuda.is_available()
            except ImportError:
                use_torch = False
        if use_torch:
            import torch
            nbytes = sc_lbm_state_bytes(self.p)
            if nbytes == 0:
                # invalid parameters: sc_lbm_create validates first and
                # returns the precise code without touching the device
                h = ctypes.c_void_p()
                _check(lib().sc_lbm_create(ctypes.byref(self.p), None, None, None, None, ctypes.byref(h)),
                       "sc_lbm_create")
                raise ScError(SC_E_INVAL, "sc_lbm_state_bytes")
            self._bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
            dev_a, dev_b = self._bufs[0].data_ptr(), self._bufs[1].data_ptr()
            if stream is None:
                stream = torch.cuda.current_stream()
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        flat = np.ascontiguousarray(rho0.transpose()).ravel()
        self.h = sc_lbm_create(self.p, flat, dev_a, dev_b, stream or None)

    def close(self):
        if getattr(self, "h", None):
            sc_lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _unflat(self, a):
        return a.reshape(self.shape[::-1]).transpose()

    def step(self, n=1, tol=0.0):
        rc, done = sc_lbm_step(self.h, n, tol)
        if rc not in (SC_OK, SC_E_NONFINITE):
            raise ScError(rc, "sc_lbm_step")
        return rc, done

    def observe(self, fields=True):
        rho = np.zeros(self.n) if fields else None
        u = np.zeros(self.dim * self.n) if fields else None
        rc, o = sc_lbm_observe(self.h, rho, u)
        out = {"obs": o.as_dict(), "rc": rc}
        if fields:
            out["rho"] = self._unflat(rho)
            out["u"] = np.stack([self._unflat(u[k * self.n:(k + 1) * self.n]) for k in range(self.dim)])
        return out

    def check(self):
        """The observables of the fused one-pass check (no fields)."""
        rc, o = sc_lbm_check(self.h)
        return {"obs": o.as_dict(), "rc": rc}

    def force(self, psi=None):
        flat = None if psi is None else np.ascontiguousarray(np.asarray(psi, np.float64).transpose()).ravel()
        F = sc_lbm_force(self.h, self.n, self.dim, flat)
        return np.stack([self._unflat(F[k * self.n:(k + 1) * self.n]) for k in range(self.dim)])

    def state(self):
        dt = np.float64 if self.p.precision == SC_FP64 else np.float32
        f = np.zeros(self.q * self.n, dtype=dt)
        sc_lbm_observe(self.h, None, None, f)
        return f

    def set_walls(self, solid, rho_w):
        """Solid mask indexed [x, y] (nonzero = solid) and virtual wall
        density; None removes the walls."""
        flat = None
        if solid is not None:
            flat = np.ascontiguousarray(np.asarray(solid).transpose()).ravel().astype(np.uint8)
        sc_lbm_set_walls(self.h, flat, rho_w)
        return self

    def set_state(self, f, step):
        sc_lbm_set_state(self.h, np.ascontiguousarray(f), step)

    @property
    def stream(self):
        """hipStream_t the library enqueues on (as an int)."""
        return lib().sc_lbm_stream(self.h)

    @property
    def rho_ref(self):
        """The storage shift the state uses (state = f - w rho_ref)."""
        return lib().sc_lbm_rho_ref(self.h)

    @property
    def variant(self):
        return sc_lbm_variant_name(self.h)

    @property
    def steps_per_launch(self):
        """Time steps one kernel launch of the current shape advances."""
        return lib().sc_lbm_steps_per_launch(self.h)


# ---------------------------------------------------------------------------
# batched sweeps
# ---------------------------------------------------------------------------

def sc_lbm_batch_create(params, rho_inits=None, stream=None):
    n = len(params)
    arr = (sc_lbm_params * n)(*params)
    keep = None
    ptrs = None
    if rho_inits is not None:
        keep = [np.ascontiguousarray(r, dtype=np.float64) for r in rho_inits]
        ptrs = (ctypes.POINTER(ctypes.c_double) * n)(*[_dptr(r) for r in keep])
    h = ctypes.c_void_p()
    rc = lib().sc_lbm_batch_create(arr, n, ptrs, stream, ctypes.byref(h))
    _check(rc, "sc_lbm_batch_create")
    return h.value


def sc_lbm_batch_step(h, max_steps, tol=0.0):
    done = ctypes.c_int64(0)
    rc = lib().sc_lbm_batch_step(h, int(max_steps), float(tol), ctypes.byref(done))
    return rc, done.value


def sc_lbm_batch_observe(h, item, rho_out=None, u_out=None):
    o = sc_lbm_obs()
    rc = lib().sc_lbm_batch_observe(h, item, ctypes.byref(o), _dptr(rho_out), _dptr(u_out))
    if rc not in (SC_OK, SC_E_NONFINITE):
        raise ScError(rc, "sc_lbm_batch_observe")
    return rc, o


def sc_lbm_batch_status(h, item):
    st, by = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().sc_lbm_batch_status(h, item, ctypes.byref(st), ctypes.byref(by)), "sc_lbm_batch_status")
    return st.value, by.value


def sc_lbm_batch_active(h):
    return lib().sc_lbm_batch_active(h)


def sc_lbm_batch_destroy(h):
    lib().sc_lbm_batch_destroy(h)


def batch_autotune(items, steps=64, **common):
    """Fastest batched launch shape for these items (dicts as for Batch):
    returns (variant, ms per step); pass variant=... to Batch to use it."""
    params = []
    for it in items:
        kw = dict(common)
        kw.update({k: v for k, v in it.items() if k != "rho0"})
        params.append(make_params("D2Q9", np.asarray(it["rho0"]).shape, **kw))
    arr = (sc_lbm_params * len(params))(*params)
    v, ms = ctypes.c_int32(), ctypes.c_double()
    _check(lib().sc_lbm_batch_autotune(arr, len(params), int(steps), ctypes.byref(v), ctypes.byref(ms)),
           "sc_lbm_batch_autotune")
    return v.value, ms.value


class Batch:
    """Many D2Q9 droplets advanced together (one launch per step).

    items: list of dicts with keys rho0 (array [x, y]) and any make_params
    keyword (order, G, tau, c0, ...).  Shared keywords go in **common."""

    def __init__(self, items, stream=None, **common):
        self.shapes = [np.asarray(it["rho0"]).shape for it in items]
        params, rhos = [], []
        for it in items:
            kw = dict(common)
            kw.update({k: v for k, v in it.items() if k != "rho0"})
            rho0 = np.asarray(it["rho0"], dtype=np.float64)
            params.append(make_params("D2Q9", rho0.shape, **kw))
            rhos.append(np.ascontiguousarray(rho0.transpose()).ravel())
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream()
            except ImportError:
                pass
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        self.n = len(items)
        self.h = sc_lbm_batch_create(params, rhos, stream or None)

    def close(self):
        if getattr(self, "h", None):
            sc_lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def step(self, n, tol=0.0):
        rc, done = sc_lbm_batch_step(self.h, n, tol)
        if rc not in (SC_OK, SC_E_NONFINITE):
            raise ScError(rc, "sc_lbm_batch_step")
        return rc, done

    def observe(self, item, fields=True):
        shape = self.shapes[item]
        nn = int(np.prod(shape))
        rho = np.zeros(nn) if fields else None
        u = np.zeros(2 * nn) if fields else None
        rc, o = sc_lbm_batch_observe(self.h, item, rho, u)
        out = {"obs": o.as_dict(), "rc": rc}
        if fields:
            un = lambda a: a.reshape(shape[::-1]).transpose()
            out["rho"] = un(rho)
            out["u"] = np.stack([un(u[:nn]), un(u[nn:])])
        return out

    def status(self, item):
        return sc_lbm_batch_status(self.h, item)

    @property
    def active(self):
        return sc_lbm_batch_active(self.h)

    def promote(self):
        """Continue in FP64 from the current FP32 states (retired items rejoin)."""
        _check(lib().sc_lbm_batch_promote(self.h), "sc_lbm_batch_promote")
        return self

    @property
    def variant(self):
        """Name of the batched launch shape in use."""
        return lib().sc_lbm_batch_variant_name(self.h).decode()

    @property
    def rho_ref(self):
        """The storage shift every item's state uses."""
        return lib().sc_lbm_batch_rho_ref(self.h)
