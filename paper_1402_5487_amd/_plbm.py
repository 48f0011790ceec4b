"""ctypes binding of libplbm (include/plbm.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
arguments into the C ABI and raises PlbmError on a non-zero status.  If the
shared library has not been built, importing this module fails loudly.
"""
import ctypes
import os

# libplbm must share torch's HIP runtime (torch owns the device memory and the
# streams it is handed).  Importing torch first loads torch's libamdhip64, so
# the library's dependency on that soname resolves to the same copy instead of
# pulling a second runtime into the process.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplbm.so")

PLBM_OK = 0
PLBM_EINVAL = -1
PLBM_ESINGULAR = -2
PLBM_EHIP = -3
PLBM_ENONFINITE = -4
PLBM_EUNSUPPORTED = -5

PLBM_BC_PERIODIC = 0
PLBM_BC_ZEROGRAD = 1

PLBM_F64, PLBM_F32, PLBM_F16DEV, PLBM_BF16DEV = 0, 1, 2, 3
PLBM_ROUND_NEAREST, PLBM_ROUND_STOCHASTIC = 0, 1
ROUNDING = {"nearest": PLBM_ROUND_NEAREST, "stochastic": PLBM_ROUND_STOCHASTIC}
STORAGE = {"f64": PLBM_F64, "f32": PLBM_F32, "f16dev": PLBM_F16DEV,
           "bf16dev": PLBM_BF16DEV}

MAX_Q1D = 8
GHOST = 3


class PlbmDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("q1d", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("v", ctypes.c_double * MAX_Q1D),
        ("c", ctypes.c_double * (MAX_Q1D * MAX_Q1D)),
        ("omega", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("theta0", ctypes.c_double),
        ("scale", ctypes.c_float * (MAX_Q1D * MAX_Q1D)),
        ("nz", ctypes.c_int32),
        ("rounding", ctypes.c_int32),
    ]


class PlbmError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = f"{what}: {strerror(status)} ({status})"
        if status == PLBM_EHIP:
            msg += ": " + lib.plbm_last_hip_error().decode()
        super().__init__(msg)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libplbm.so is not built ({LIB_PATH}); run "
            "`python -c 'import __graft_entry__ as g; g.build()'` first")
    lib = ctypes.CDLL(LIB_PATH)
    D = ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER(PlbmDesc)
    vp = ctypes.c_void_p
    lib.plbm_coeffs.argtypes = [ctypes.c_int, D, D]
    lib.plbm_desc_default.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int]
    lib.plbm_buffer_elems.argtypes = [P]
    lib.plbm_buffer_elems.restype = ctypes.c_size_t
    lib.plbm_elem_bytes.argtypes = [P]
    lib.plbm_elem_bytes.restype = ctypes.c_size_t
    lib.plbm_init.argtypes = [P, vp, vp, vp, vp, vp, vp]
    lib.plbm_step.argtypes = [P, vp, vp, ctypes.c_int, D, vp]
    lib.plbm_step_noalloc.argtypes = [P, vp, vp, ctypes.c_int, D, vp]
    lib.plbm_step_fields.argtypes = [P, vp, vp, ctypes.c_int, vp, vp, vp, vp, vp]
    lib.plbm_moments.argtypes = [P, vp, vp, vp, vp, vp, D, vp]
    lib.plbm_dev_scales.argtypes = [P, vp, vp, vp, vp, vp]
    lib.plbm_init3.argtypes = [P, vp, vp, vp, vp, vp, vp, vp]
    lib.plbm_moments3.argtypes = [P, vp, vp, vp, vp, vp, vp, D, vp]
    lib.plbm_strerror.argtypes = [ctypes.c_int]
    lib.plbm_strerror.restype = ctypes.c_char_p
    lib.plbm_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.plbm_last_hip_error.argtypes = []
    lib.plbm_last_hip_error.restype = ctypes.c_char_p
    return lib


lib = _load()

#: every symbol declared in include/plbm.h
EXPORTED = ("plbm_coeffs", "plbm_desc_default", "plbm_buffer_elems",
            "plbm_elem_bytes", "plbm_init", "plbm_step", "plbm_moments",
            "plbm_dev_scales", "plbm_strerror", "plbm_last_hip_error",
            "plbm_stream_copy", "plbm_init3", "plbm_moments3", "plbm_step_noalloc",
            "plbm_step_fields")


def strerror(status):
    return lib.plbm_strerror(int(status)).decode()


def check(status, what):
    if status != PLBM_OK:
        raise PlbmError(status, what)


def coeffs(v):
    """plbm_coeffs: c[i][j] for the velocity list v (host, FP64)."""
    q = len(v)
    va = (ctypes.c_double * max(q, 1))(*[float(x) for x in v])
    ca = (ctypes.c_double * max(q * q, 1))()
    check(lib.plbm_coeffs(q, va, ca), "plbm_coeffs")
    return [[ca[i * q + j] for j in range(q)] for i in range(q)]


def desc_default(dim, nx, ny, omega, storage):
    d = PlbmDesc()
    check(lib.plbm_desc_default(ctypes.byref(d), dim, nx, ny, float(omega),
                                STORAGE.get(storage, storage)), "plbm_desc_default")
    return d


def desc_q3(dim, nx, ny, omega, storage, zeta=3.0, a=1):
    """Descriptor of the isothermal three-velocity family (Eq. 1d3v): D1Q3
    with zero-gradient ends (dim 1) or its tensor product D2Q9 (dim 2,
    periodic); velocities (0, +a, -a), reference temperature
    theta0 = a^2 / zeta, table from plbm_coeffs."""
    d = desc_default(dim, nx, ny, omega, storage)
    v = [0.0, float(a), -float(a)]
    c = coeffs(v)
    d.q1d = 3
    for i in range(len(d.v)):
        d.v[i] = v[i] if i < 3 else 0.0
    for i in range(len(d.c)):
        d.c[i] = c[i // 3][i % 3] if i < 9 else 0.0
    d.theta0 = float(a) * float(a) / float(zeta)
    return d


def desc_general(dim, nx, ny, omega, storage, v, theta0=None):
    """Descriptor for any on-lattice 1D velocity set v (3 to 7 distinct
    integers, |v| <= 3; Sec. 2.2), table from plbm_coeffs.  Sets of up to
    four velocities are isothermal models at theta0 (required), larger sets
    thermal.  dim 1: zero-gradient ends; dim 2: tensor product, periodic."""
    q = len(v)
    if q <= 4 and theta0 is None:
        raise ValueError("sets of up to four velocities are isothermal: give theta0")
    d = desc_default(dim, nx, ny, omega, storage)
    c = coeffs(v)
    d.q1d = q
    for i in range(len(d.v)):
        d.v[i] = float(v[i]) if i < q else 0.0
    for i in range(len(d.c)):
        d.c[i] = c[i // q][i % q] if i < q * q else 0.0
    if theta0 is not None:
        d.theta0 = float(theta0)
    if buffer_elems(d) == 0:
        raise PlbmError(PLBM_EINVAL, "desc_general")
    return d


def desc_3d(nx, ny, nz, omega, storage):
    """Descriptor of the D3Q125 model (dim 3, periodic): the D1Q5 set
    {0, +-1, +-3} along each axis, depth nz."""
    d = desc_default(3, nx, ny, omega, storage)
    d.nz = int(nz)
    if buffer_elems(d) == 0:
        raise PlbmError(PLBM_EINVAL, "desc_3d")
    return d


def buffer_elems(d):
    return int(lib.plbm_buffer_elems(ctypes.byref(d)))


def elem_bytes(d):
    return int(lib.plbm_elem_bytes(ctypes.byref(d)))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    return ctypes.c_void_p(stream)


def init(d, rho, ux, uy, theta, f, stream):
    check(lib.plbm_init(ctypes.byref(d), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(theta),
                        _ptr(f), _stream(stream)), "plbm_init")


def step(d, fa, fb, nsteps, want_sums, stream):
    sums = (ctypes.c_double * (5 if d.dim == 3 else 4))() if want_sums else None
    check(lib.plbm_step(ctypes.byref(d), _ptr(fa), _ptr(fb), int(nsteps), sums,
                        _stream(stream)), "plbm_step")
    return list(sums) if want_sums else None


def step_fields(d, fa, fb, nsteps, rho, ux, uy, theta, stream):
    """plbm_step_fields: nsteps steps, the first also writing the fields
    of the state it reads into the given FP64 device tensors (or None)."""
    check(lib.plbm_step_fields(ctypes.byref(d), _ptr(fa), _ptr(fb), int(nsteps), _ptr(rho), _ptr(ux),
                               _ptr(uy), _ptr(theta), _stream(stream)), "plbm_step_fields")


def step_noalloc(d, fa, fb, nsteps, want_sums, stream):
    """plbm_step_noalloc: as step(), with the sums' partials in the
    library's static device scratch instead of an allocation."""
    sums = (ctypes.c_double * 4)() if want_sums else None
    check(lib.plbm_step_noalloc(ctypes.byref(d), _ptr(fa), _ptr(fb), int(nsteps), sums,
                                _stream(stream)), "plbm_step_noalloc")
    return list(sums) if want_sums else None


def moments(d, f, rho, ux, uy, theta, want_sums, stream):
    sums = (ctypes.c_double * 4)() if want_sums else None
    check(lib.plbm_moments(ctypes.byref(d), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy),
                           _ptr(theta), sums, _stream(stream)), "plbm_moments")
    return list(sums) if want_sums else None


def init3(d, rho, ux, uy, uz, theta, f, stream):
    check(lib.plbm_init3(ctypes.byref(d), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz), _ptr(theta),
                         _ptr(f), _stream(stream)), "plbm_init3")


def moments3(d, f, rho, ux, uy, uz, theta, want_sums, stream):
    sums = (ctypes.c_double * 5)() if want_sums else None
    check(lib.plbm_moments3(ctypes.byref(d), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(uz),
                            _ptr(theta), sums, _stream(stream)), "plbm_moments3")
    return list(sums) if want_sums else None


def dev_scales(d, rho, ux, uy, theta, stream):
    check(lib.plbm_dev_scales(ctypes.byref(d), _ptr(rho), _ptr(ux), _ptr(uy),
                              _ptr(theta), _stream(stream)), "plbm_dev_scales")


def step_vjp(d, post, lam, out, stream):
    """plbm_step_vjp: out = dL/dpost for the step that read `post`, given
    lam = dL/d(the buffer it wrote) (FP64 adjoint buffers)."""
    check(lib.plbm_step_vjp(ctypes.byref(d), _ptr(post), _ptr(lam), _ptr(out), _stream(stream)),
          "plbm_step_vjp")


def stream_copy(src, dst, nbytes, stream):
    """plbm_stream_copy: the HBM calibration copy."""
    check(lib.plbm_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)),
          "plbm_stream_copy")


# ---------------------------------------------------------------------------
# batching form
# ---------------------------------------------------------------------------
class LatticeSpec(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("omega", ctypes.c_double)]


BATCH_MAX_CLASSES = 32


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("grid_mode", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("parity", ctypes.c_int32),
                ("nodes", ctypes.c_int64), ("pool_bytes", ctypes.c_int64),
                ("classes", ctypes.c_int32),
                ("class_size", ctypes.c_int32 * BATCH_MAX_CLASSES),
                ("class_w", ctypes.c_int32 * BATCH_MAX_CLASSES),
                ("class_r", ctypes.c_int32 * BATCH_MAX_CLASSES)]


def _setup_batch(lib):
    vp, P = ctypes.c_void_p, ctypes.POINTER(PlbmDesc)
    lib.plbm_batch_create.argtypes = [P, ctypes.POINTER(LatticeSpec), ctypes.c_int,
                                      ctypes.POINTER(vp)]
    lib.plbm_batch_destroy.argtypes = [vp]
    lib.plbm_batch_init.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
    lib.plbm_batch_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    lib.plbm_batch_set_graph_steps.argtypes = [vp, ctypes.c_int]
    lib.plbm_batch_step.argtypes = [vp, ctypes.c_int, vp]
    lib.plbm_batch_moments.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp,
                                       ctypes.POINTER(ctypes.c_double), vp]
    lib.plbm_batch_lattice.argtypes = [vp, ctypes.c_int, P, ctypes.POINTER(vp)]
    lib.plbm_batch_query.argtypes = [vp, ctypes.POINTER(BatchInfo)]


_setup_batch(lib)
EXPORTED = EXPORTED + ("plbm_batch_create", "plbm_batch_destroy", "plbm_batch_init",
                       "plbm_batch_autotune", "plbm_batch_set_graph_steps",
                       "plbm_batch_step", "plbm_batch_moments", "plbm_batch_lattice",
                       "plbm_batch_query")


# ---------------------------------------------------------------------------
# learned closure
# ---------------------------------------------------------------------------
CNN_LAYER_PARAMS = 9248
CNN_PARAMS = 3 * CNN_LAYER_PARAMS


def _setup_closure(lib):
    vp, P = ctypes.c_void_p, ctypes.POINTER(PlbmDesc)
    F = ctypes.POINTER(ctypes.c_float)
    lib.plbm_closure_create.argtypes = [P, ctypes.c_int, ctypes.POINTER(vp)]
    lib.plbm_closure_destroy.argtypes = [vp]
    lib.plbm_closure_set_norm.argtypes = [vp, F, F, F, F]
    lib.plbm_closure_forward.argtypes = [vp, vp, ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_float,
                                         vp]
    lib.plbm_closure_backward.argtypes = [vp, vp, ctypes.POINTER(vp), ctypes.c_float, vp,
                                          ctypes.POINTER(ctypes.c_double), vp]
    lib.plbm_closure_adam.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
    lib.plbm_closure_apply.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, ctypes.c_float, vp, vp]
    lib.plbm_closure_activation.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp),
                                            ctypes.POINTER(ctypes.c_size_t)]
    lib.plbm_restrict.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  vp, vp, vp, vp, vp]
    lib.plbm_closure_target.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, vp, vp]
    D = ctypes.POINTER(ctypes.c_double)
    lib.plbm_step_vjp.argtypes = [P, vp, vp, vp, vp]
    lib.plbm_closure_rollout_loss.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int,
                                              ctypes.c_double, ctypes.POINTER(vp), D, vp]
    lib.plbm_closure_apply_vjp.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.plbm_closure_backward_vjp.argtypes = [vp, vp, ctypes.c_float, vp, ctypes.c_int,
                                              ctypes.POINTER(vp), vp]
    lib.plbm_closure_rollout_vjp.argtypes = [vp, P, vp, ctypes.c_float, vp, ctypes.c_int,
                                             ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double,
                                             ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                             ctypes.POINTER(vp), ctypes.c_int, D, vp]


_setup_closure(lib)
EXPORTED = EXPORTED + ("plbm_closure_create", "plbm_closure_destroy", "plbm_closure_set_norm",
                       "plbm_closure_forward", "plbm_closure_backward", "plbm_closure_adam",
                       "plbm_closure_apply", "plbm_closure_activation", "plbm_closure_target",
                       "plbm_restrict", "plbm_step_vjp", "plbm_closure_rollout_loss",
                       "plbm_closure_apply_vjp", "plbm_closure_backward_vjp",
                       "plbm_closure_rollout_vjp")
