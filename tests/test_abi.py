"""CPU tests of the C ABI: the library loads, exports every declared symbol,
its host-side coefficient table agrees with the oracle, and argument
validation rejects bad calls before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1402_5487_amd import _plbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(plbm_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    declared = _declared()
    assert "plbm_step" in declared and "plbm_coeffs" in declared
    for name in declared:
        assert hasattr(_plbm.lib, name), name
    assert set(declared) <= set(_plbm.EXPORTED) | set(getattr(_plbm, "EXPORTED_EXTRA", ()))


@pytest.mark.parametrize("v", [(0, 1, -1, 3, -3), (0, 1, -1, 2, -2), (0, 2, -4),
                               (1, -1, 3, -3), (0, 1, -1, 3, -3, 5, -5), (0.0, 1.4, -1.4, 2.8, -2.8)])
def test_coeffs_match_oracle(v):
    got = np.array(_plbm.coeffs(v))
    ref = oracle.lagrange_coeffs(v)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_coeffs_errors():
    with pytest.raises(_plbm.PlbmError) as e:
        _plbm.coeffs((0, 1, 1))
    assert e.value.status == _plbm.PLBM_ESINGULAR
    with pytest.raises(_plbm.PlbmError) as e:
        _plbm.coeffs(tuple(range(9)))
    assert e.value.status == _plbm.PLBM_EINVAL
    assert _plbm.lib.plbm_coeffs(5, None, None) == _plbm.PLBM_EINVAL
    assert _plbm.lib.plbm_coeffs(0, None, None) == _plbm.PLBM_EINVAL


def test_desc_defaults_and_sizes():
    d = _plbm.desc_default(2, 100, 60, 1.8, "f32")
    assert d.q1d == 5 and d.bc == _plbm.PLBM_BC_PERIODIC
    assert list(d.v)[:5] == [0, 1, -1, 3, -3]
    assert _plbm.buffer_elems(d) == 25 * 100 * 60
    assert _plbm.elem_bytes(d) == 4
    d1 = _plbm.desc_default(1, 1000, 1, 1.0, "f64")
    assert d1.bc == _plbm.PLBM_BC_ZEROGRAD
    assert _plbm.buffer_elems(d1) == 5 * (1000 + 6)
    assert _plbm.elem_bytes(d1) == 8


@pytest.mark.parametrize("dim,nx,ny,omega,storage", [
    (4, 10, 10, 1.0, "f64"), (0, 10, 10, 1.0, "f64"), (2, 0, 10, 1.0, "f64"), (2, 10, 10, 0.0, "f64"),
    (2, 10, 10, 2.0, "f64"), (2, 2, 10, 1.0, "f64"), (2, 10, 10, 1.0, 7)])
def test_desc_rejects(dim, nx, ny, omega, storage):
    with pytest.raises(_plbm.PlbmError) as e:
        _plbm.desc_default(dim, nx, ny, omega, storage)
    assert e.value.status == _plbm.PLBM_EINVAL


def test_step_validates_before_launch():
    d = _plbm.desc_default(2, 64, 64, 1.5, "f64")
    buf = ctypes.c_void_p(0x1000)
    lib = _plbm.lib
    # aliasing buffers, null buffers, negative step count, bad omega
    assert lib.plbm_step(ctypes.byref(d), buf, buf, 1, None, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step(ctypes.byref(d), None, buf, 1, None, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step(ctypes.byref(d), buf, ctypes.c_void_p(0x2000), -1, None,
                         None) == _plbm.PLBM_EINVAL
    d.omega = 2.5
    assert lib.plbm_step(ctypes.byref(d), buf, ctypes.c_void_p(0x2000), 1, None,
                         None) == _plbm.PLBM_EINVAL
    d.omega = 1.5
    d.v[1] = 0.5      # off-lattice velocity cannot stream
    assert lib.plbm_step(ctypes.byref(d), buf, ctypes.c_void_p(0x2000), 1, None,
                         None) == _plbm.PLBM_EINVAL
    d.v[1] = 4.0      # beyond the three ghost/halo nodes
    assert lib.plbm_step(ctypes.byref(d), buf, ctypes.c_void_p(0x2000), 1, None,
                         None) == _plbm.PLBM_EINVAL
    d.v[1] = 1.0
    d.q1d = 3         # valid descriptor, kernels compiled for five velocities
    d.v[0], d.v[1], d.v[2] = 0.0, 1.0, -1.0
    assert lib.plbm_step(ctypes.byref(d), buf, ctypes.c_void_p(0x2000), 1, None,
                         None) == _plbm.PLBM_EUNSUPPORTED


def test_step_noalloc_validates_before_launch():
    """The allocation-free step refuses, before any device call, the models it
    does not take and a 1D lattice with sums whose partials exceed its
    scratch (8192 workgroups of 256 nodes)."""
    lib = _plbm.lib
    a, b = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    s = (ctypes.c_double * 4)()
    d = _plbm.desc_default(2, 64, 64, 1.5, "f64")
    assert lib.plbm_step_noalloc(ctypes.byref(d), a, a, 1, s, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step_noalloc(ctypes.byref(d), a, b, -1, s, None) == _plbm.PLBM_EINVAL
    d1 = _plbm.desc_default(1, 8192 * 256 + 1, 1, 1.0, "f64")
    assert lib.plbm_step_noalloc(ctypes.byref(d1), a, b, 1, s, None) == _plbm.PLBM_EINVAL
    q9 = _plbm.desc_q3(2, 64, 64, 1.5, "f64", zeta=4.0)
    assert lib.plbm_step_noalloc(ctypes.byref(q9), a, b, 1, s, None) == _plbm.PLBM_EUNSUPPORTED
    d3 = _plbm.desc_3d(16, 16, 16, 1.5, "f64")
    assert lib.plbm_step_noalloc(ctypes.byref(d3), a, b, 1, s, None) == _plbm.PLBM_EUNSUPPORTED
    dg = _plbm.desc_general(2, 64, 64, 1.5, "f64", (0, 1, -1, 2, -3), theta0=None)
    assert lib.plbm_step_noalloc(ctypes.byref(dg), a, b, 1, s, None) == _plbm.PLBM_EUNSUPPORTED


def test_step_fields_and_rollout_vjp_validate_before_launch():
    """plbm_step_fields takes D2Q25 only and at least one step; the fused
    rollout adjoint refuses a missing closure or arrays before any device
    call."""
    lib = _plbm.lib
    a, b = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    d = _plbm.desc_default(2, 64, 64, 1.5, "f64")
    assert lib.plbm_step_fields(ctypes.byref(d), a, b, 0, None, None, None, None, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step_fields(ctypes.byref(d), a, a, 1, None, None, None, None, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step_fields(None, a, b, 1, None, None, None, None, None) == _plbm.PLBM_EINVAL
    for other in (_plbm.desc_default(1, 64, 1, 1.0, "f64"), _plbm.desc_q3(2, 64, 64, 1.5, "f64", zeta=4.0),
                  _plbm.desc_3d(16, 16, 16, 1.5, "f64"),
                  _plbm.desc_general(2, 64, 64, 1.5, "f64", (0, 1, -1, 2, -3))):
        assert lib.plbm_step_fields(ctypes.byref(other), a, b, 1, None, None, None, None,
                                    None) == _plbm.PLBM_EUNSUPPORTED
    p = ctypes.c_void_p(0x3000)
    arr = (ctypes.c_void_p * 1)(0x4000)
    assert lib.plbm_closure_rollout_vjp(None, ctypes.byref(d), p, 0.0, p, 0, arr, arr, 1.0, arr, None, None,
                                        None, 1, None, None) == _plbm.PLBM_EINVAL


def test_general_sets_are_validated_before_launch():
    """Asymmetric and q1d = 4, 6, 7 sets take the general kernels; what they
    cannot run is refused on the host: 16-bit storage, a table that is not
    the Lagrange table of v, an isothermal set without theta0, q1d = 8."""
    buf, other = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    lib = _plbm.lib
    d = _plbm.desc_general(2, 64, 64, 1.5, "f64", (0, 1, -1, 2, -3))
    assert _plbm.buffer_elems(d) == 25 * 64 * 64
    d.storage = _plbm.PLBM_F16DEV
    assert lib.plbm_step(ctypes.byref(d), buf, other, 1, None, None) == _plbm.PLBM_EUNSUPPORTED
    d = _plbm.desc_general(2, 64, 64, 1.5, "f64", (0, 1, -1, 2, -3))
    d.c[7] += 1e-3                     # no longer the Lagrange table of v
    assert lib.plbm_step(ctypes.byref(d), buf, other, 1, None, None) == _plbm.PLBM_EINVAL
    d = _plbm.desc_general(1, 100, 1, 1.0, "f32", (1, -1, 3, -3), theta0=4 / 3)
    assert _plbm.buffer_elems(d) == 4 * (100 + 6)
    d.theta0 = 0.0                     # isothermal sets need their theta0
    assert lib.plbm_step(ctypes.byref(d), buf, other, 1, None, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step(ctypes.byref(d), buf, buf, 1, None, None) == _plbm.PLBM_EINVAL
    with pytest.raises(ValueError):
        _plbm.desc_general(2, 64, 64, 1.5, "f64", (1, -1, 3, -3))
    d = _plbm.desc_general(2, 64, 64, 1.5, "f64", (0, 1, -1, 2, -2, 3, -3))
    d.q1d = 8                          # eight distinct velocities cannot fit |v| <= 3
    d.v[7] = 3.0
    assert lib.plbm_step(ctypes.byref(d), buf, other, 1, None, None) != _plbm.PLBM_OK


def test_dev_scales_must_be_powers_of_two_per_class():
    d = _plbm.desc_default(2, 64, 64, 1.5, "f16dev")
    buf = ctypes.c_void_p(0x1000)
    d.scale[0] = 0.3     # not a power of two
    assert _plbm.lib.plbm_step(ctypes.byref(d), buf, ctypes.c_void_p(0x2000), 1, None,
                               None) == _plbm.PLBM_EINVAL
    d.scale[0] = 1.0
    d.scale[1] = 0.5     # k = 1 and k = 2 share a class (|v_x| = 1, v_y = 0)
    assert _plbm.lib.plbm_step(ctypes.byref(d), buf, ctypes.c_void_p(0x2000), 1, None,
                               None) == _plbm.PLBM_EINVAL


def test_dev_storage_rejected_in_1d():
    d = _plbm.desc_default(1, 100, 1, 1.0, "f64")
    d.storage = _plbm.PLBM_F16DEV
    assert _plbm.lib.plbm_init(ctypes.byref(d), ctypes.c_void_p(8), ctypes.c_void_p(8),
                               None, ctypes.c_void_p(8), ctypes.c_void_p(8),
                               None) == _plbm.PLBM_EUNSUPPORTED


def test_node_count_limit():
    """Every form keeps its node count within 2^30 (1D included: its grid
    sizes are computed in 32-bit integers)."""
    d = _plbm.desc_default(1, 1 << 30, 1, 1.0, "f64")
    assert _plbm.buffer_elems(d) == 5 * ((1 << 30) + 6)
    d.nx = (1 << 30) + 1
    assert _plbm.buffer_elems(d) == 0
    d = _plbm.desc_default(2, 1 << 15, 1 << 15, 1.0, "f64")
    assert _plbm.buffer_elems(d) == 25 << 30
    d.ny += 1
    assert _plbm.buffer_elems(d) == 0


def test_rounding_mode_validation():
    """Stochastic rounding applies to the 16-bit deviation forms only."""
    buf, other = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    d = _plbm.desc_default(2, 64, 64, 1.5, "f16dev")
    d.rounding = _plbm.PLBM_ROUND_STOCHASTIC
    assert _plbm.buffer_elems(d) == 25 * 64 * 64
    d.rounding = 2
    assert _plbm.buffer_elems(d) == 0
    d = _plbm.desc_default(2, 64, 64, 1.5, "f32")
    d.rounding = _plbm.PLBM_ROUND_STOCHASTIC
    assert _plbm.lib.plbm_step(ctypes.byref(d), buf, other, 1, None, None) == _plbm.PLBM_EINVAL


def test_strerror():
    assert _plbm.strerror(0) == "ok"
    assert "non-finite" in _plbm.strerror(_plbm.PLBM_ENONFINITE)
    assert _plbm.strerror(-99) == "unknown status"


def test_three_velocity_family_descriptor_and_rejections():
    """q1d = 3 (isothermal D2Q9): a valid descriptor sizes 9 populations per
    node; 16-bit storage and asymmetric sets are refused before launch, and a
    1D descriptor must keep its zero-gradient ends."""
    d = _plbm.desc_q3(2, 64, 32, 1.8, "f64", zeta=4.0)
    assert d.q1d == 3 and abs(d.theta0 - 0.25) < 1e-15
    assert _plbm.buffer_elems(d) == 9 * 64 * 32
    buf = ctypes.c_void_p(16)         # never dereferenced: validation fails first
    other = ctypes.c_void_p(32)
    for change in ("f16", "dim1", "asym"):
        e = _plbm.desc_q3(2, 64, 32, 1.8, "f64", zeta=4.0)
        if change == "f16":
            e.storage = _plbm.PLBM_F16DEV
            for k in range(9):
                e.scale[k] = 1.0
        elif change == "dim1":
            e.dim, e.ny, e.bc = 1, 1, 0
        else:
            # an asymmetric set goes to the general kernels, which check the
            # table against v: the symmetric table of (0, 1, -1) is refused
            e.v[2] = -2.0
        rc = _plbm.lib.plbm_step(ctypes.byref(e), buf, other, 1, None, None)
        want = {"f16": _plbm.PLBM_EUNSUPPORTED, "dim1": _plbm.PLBM_EINVAL,
                "asym": _plbm.PLBM_EINVAL}[change]
        assert rc == want, (change, rc)
    d1 = _plbm.desc_q3(1, 1000, 1, 0.93, "f64", zeta=4.0)
    assert _plbm.buffer_elems(d1) == 3 * (1000 + 6)


def test_d3q125_descriptor_and_rejections():
    """dim 3 (D3Q125, Sec. 2.4): 125 populations per node, depth nz; 16-bit
    storage, a depth below the largest shift, a 2D descriptor with a depth,
    and the 2D entry points are refused before any device work."""
    d = _plbm.desc_3d(40, 20, 10, 1.5, "f32")
    assert d.dim == 3 and d.nz == 10 and d.bc == _plbm.PLBM_BC_PERIODIC
    assert _plbm.buffer_elems(d) == 125 * 40 * 20 * 10 and _plbm.elem_bytes(d) == 4
    assert _plbm.desc_default(3, 16, 12, 1.0, "f64").nz == 12      # nz defaults to ny
    with pytest.raises(_plbm.PlbmError) as e:
        _plbm.desc_3d(40, 20, 10, 1.5, "f16dev")
    assert e.value.status == _plbm.PLBM_EUNSUPPORTED
    for nz in (0, 2):
        with pytest.raises(_plbm.PlbmError):
            _plbm.desc_3d(40, 20, nz, 1.5, "f64")
    d2 = _plbm.desc_default(2, 40, 20, 1.5, "f64")
    d2.nz = 4
    assert _plbm.buffer_elems(d2) == 0
    lib, p, q = _plbm.lib, ctypes.c_void_p(16), ctypes.c_void_p(32)
    d = _plbm.desc_3d(40, 20, 10, 1.5, "f64")
    assert lib.plbm_init(ctypes.byref(d), p, p, p, p, q, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_moments(ctypes.byref(d), q, None, None, None, None, None,
                            None) == _plbm.PLBM_EINVAL
    assert lib.plbm_init3(ctypes.byref(d), p, p, None, p, p, q, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step(ctypes.byref(d), p, p, 1, None, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_step(ctypes.byref(d), p, q, -1, None, None) == _plbm.PLBM_EINVAL
    d2 = _plbm.desc_default(2, 40, 20, 1.5, "f64")
    assert lib.plbm_init3(ctypes.byref(d2), p, p, p, p, p, q, None) == _plbm.PLBM_EINVAL
    assert lib.plbm_moments3(ctypes.byref(d2), q, None, None, None, None, None, None,
                             None) == _plbm.PLBM_EINVAL
    # rows whose population rows could not be addressed with 32-bit offsets
    d = _plbm.desc_3d(40, 20, 10, 1.5, "f64")
    d.nx, d.ny, d.nz = (1 << 26) + 1, 3, 3
    assert _plbm.buffer_elems(d) == 0

