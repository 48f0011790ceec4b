"""plbm_step_noalloc against plbm_step, through the C ABI.

The allocation-free entry point keeps the partial sums of its sums launch in
the library's static device scratch.  Its populations must equal plbm_step's
bitwise (same per-node arithmetic) and its FP64 sums agree to rounding (their
partials are grouped differently).  Each case makes two calls in a row, the
second on a smaller lattice, so that whatever the first call left in the
shared scratch cannot leak into the second.
"""
import ctypes

import numpy as np
import pytest

from paper_1402_5487_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(dim, nx, ny, storage, seed):
    from paper_1402_5487_amd.lattice import Lattice
    if dim == 2:
        fields = inputs.random_fields(nx, ny, seed=seed)
    else:
        fields = inputs.shock_tube(nx, rho_r=0.5)
    lat = Lattice(dim, nx, ny, omega=1.8 if dim == 2 else 1.0, storage=storage,
                  theta0=0.35 if storage != "f64" else None).init(*fields)
    return lat


def _call(fn, lat, fa, fb, nsteps, want_sums):
    from paper_1402_5487_amd import _plbm
    sums = (ctypes.c_double * 4)() if want_sums else None
    rc = fn(ctypes.byref(lat.desc), ctypes.c_void_p(fa.data_ptr()),
            ctypes.c_void_p(fb.data_ptr()), int(nsteps), sums,
            ctypes.c_void_p(lat.stream))
    assert rc == _plbm.PLBM_OK, _plbm.strerror(rc)
    return np.array(list(sums)) if want_sums else None


def _compare(lat, nsteps):
    import torch
    from paper_1402_5487_amd import _plbm
    a0, a1 = lat.f.clone(), torch.empty_like(lat.f)
    b0, b1 = lat.f.clone(), torch.empty_like(lat.f)
    s_ref = _call(_plbm.lib.plbm_step, lat, a0, a1, nsteps, True)
    s_new = _call(_plbm.lib.plbm_step_noalloc, lat, b0, b1, nsteps, True)
    torch.cuda.synchronize()
    out_a = a0 if nsteps % 2 == 0 else a1
    out_b = b0 if nsteps % 2 == 0 else b1
    assert torch.equal(out_a.view(torch.uint8), out_b.view(torch.uint8)), \
        f"populations differ ({lat.nx}x{lat.ny}, {nsteps} steps)"
    # the invariants of a KH or shock-tube state are O(nodes); FP64 partial sums
    # regrouped over at most 8192 + 2^22 terms agree far below 1e-12 relative
    scale = np.abs(s_ref).max()
    assert np.abs(s_new - s_ref).max() <= 1e-12 * scale, (s_new, s_ref)
    return s_ref


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_noalloc_matches_step_2d_two_calls(storage):
    # first call: 1024 x 2100 nodes = 8400 row tiles, more than the scratch's
    # 8192 workgroups, so the capped grid walks several tiles per workgroup;
    # second call: a smaller ragged lattice
    print(f"noalloc 2D {storage}: 1024x2100 then 300x37", flush=True)
    _compare(_pair(2, 1024, 2100, storage, seed=11), 3)
    _compare(_pair(2, 300, 37, storage, seed=12), 4)


def test_noalloc_matches_step_1d_two_calls():
    print("noalloc 1D: 1000 then 130 nodes", flush=True)
    _compare(_pair(1, 1000, 1, "f64", seed=0), 5)
    _compare(_pair(1, 130, 1, "f64", seed=0), 2)


def test_noalloc_without_sums_and_zero_steps():
    import torch
    from paper_1402_5487_amd import _plbm
    lat = _pair(2, 257, 40, "f64", seed=3)
    a0, a1 = lat.f.clone(), torch.empty_like(lat.f)
    b0, b1 = lat.f.clone(), torch.empty_like(lat.f)
    _call(_plbm.lib.plbm_step, lat, a0, a1, 3, False)
    _call(_plbm.lib.plbm_step_noalloc, lat, b0, b1, 3, False)
    torch.cuda.synchronize()
    assert torch.equal(a1, b1)
    # zero steps with sums: the invariants of the current state
    s_ref = lat.sums()
    s_new = _call(_plbm.lib.plbm_step_noalloc, lat, lat.f, a0, 0, True)
    assert np.abs(s_new - np.array(s_ref)).max() <= 1e-12 * np.abs(s_ref).max()


def test_noalloc_rejects_what_it_does_not_take():
    import torch
    from paper_1402_5487_amd import _plbm
    from paper_1402_5487_amd.lattice import Lattice
    q9 = Lattice(2, 64, 8, omega=1.2, storage="f64", zeta=4.0)
    buf = torch.zeros(4, dtype=torch.float64, device="cuda")
    s = (ctypes.c_double * 4)()
    for desc in (q9.desc, _plbm.desc_3d(16, 16, 16, 1.2, "f64")):
        rc = _plbm.lib.plbm_step_noalloc(ctypes.byref(desc), ctypes.c_void_p(buf.data_ptr()),
                                         ctypes.c_void_p(buf.data_ptr() + 8), 1, s, None)
        assert rc == _plbm.PLBM_EUNSUPPORTED
    # a 1D lattice with more than 8192 * 256 nodes cannot keep its partials
    d = _plbm.desc_default(1, 8192 * 256 + 1, 1, 1.0, "f64")
    rc = _plbm.lib.plbm_step_noalloc(ctypes.byref(d), ctypes.c_void_p(buf.data_ptr()),
                                     ctypes.c_void_p(buf.data_ptr() + 8), 1, s, None)
    assert rc == _plbm.PLBM_EINVAL
