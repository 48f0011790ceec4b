"""GPU parity of the general-velocity-set kernels (Sec. 2.2: any on-lattice
set through Eq. rdr) against the FP64 oracle: D1Q4 / D2Q16, asymmetric
three- and five-velocity sets, q1d = 6 and 7, in 1D and 2D."""
import numpy as np
import pytest
import torch

import oracle
from helpers import rel_err
from paper_1402_5487_amd import inputs
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24

# name: (velocities, temperature, isothermal)
SETS = {
    "d1q4": ([1, -1, 3, -3], 4.0 / 3.0, True),
    "q3_asym": ([0, 1, -2], 0.25, True),
    "q5_asym": ([0, 1, -1, 2, -3], 0.7, False),
    "q6": ([0, 1, -1, 2, -2, 3], 0.5, False),
    "q7": ([0, 1, -1, 2, -2, 3, -3], 1.0, False),
}


def _fields2(nx, ny, th, seed):
    rng = np.random.default_rng(seed)
    shp = (ny, nx)
    return (1 + 0.02 * rng.uniform(-1, 1, shp), 0.03 * rng.uniform(-1, 1, shp),
            0.03 * rng.uniform(-1, 1, shp), th * (1 + 0.02 * rng.uniform(-1, 1, shp)))


def _gpu(name, dim, nx, ny, omega, storage="f64"):
    v, th, iso = SETS[name]
    return Lattice(dim, nx, ny, omega=omega, storage=storage, velocities=v,
                   theta0=th if iso else None)


def _ref(name, dim, nx, ny, omega):
    v, th, iso = SETS[name]
    return oracle.Lattice(dim, nx, ny, v=v, omega=omega, bc=1 if dim == 1 else 0,
                          theta0=th if iso else None)


def _pulled2(lat, v):
    q = len(v)
    a = lat.f.double().cpu().numpy().reshape(lat.ny, q * q, lat.nx).transpose(1, 0, 2)
    out = np.empty_like(a)
    for k in range(q * q):
        out[k] = np.roll(a[k], (v[k // q], v[k % q]), axis=(0, 1))
    return out


@pytest.mark.parametrize("name", sorted(SETS))
@pytest.mark.parametrize("nx,ny,steps", [(7, 5, 16), (300, 37, 20)])
def test_step2d_f64_matches_oracle(name, nx, ny, steps):
    v, th, _ = SETS[name]
    fields = _fields2(nx, ny, th, seed=nx + len(v))
    lat = _gpu(name, 2, nx, ny, 1.4).init(*fields)
    lat.step(steps)
    got = [t.cpu().numpy() for t in lat.moments()]
    ref = _ref(name, 2, nx, ny, 1.4)
    f = ref.step(ref.init(*fields), steps)
    want = ref.moments(f)
    assert rel_err(got[0], want[0]) < 1e-12
    assert max(rel_err(got[1], want[1], 0.03), rel_err(got[2], want[2], 0.03)) < 1e-12
    assert rel_err(got[3], want[3]) < 1e-12
    assert rel_err(_pulled2(lat, v), f) < 1e-12


@pytest.mark.parametrize("name", sorted(SETS))
def test_init_then_moments(name):
    v, th, iso = SETS[name]
    fields = _fields2(40, 9, th, seed=1)
    lat = _gpu(name, 2, 40, 9, 1.2).init(*fields)
    rho, ux, uy, tt = (t.cpu().numpy() for t in lat.moments())
    assert rel_err(rho, fields[0]) < 1e-14
    assert max(rel_err(ux, fields[1], 0.03), rel_err(uy, fields[2], 0.03)) < 1e-13
    assert rel_err(tt, np.full_like(tt, th) if iso else fields[3]) < 1e-13


@pytest.mark.parametrize("name", sorted(SETS))
@pytest.mark.parametrize("n", [1, 5, 300])
def test_step1d_f64_matches_oracle(name, n):
    v, th, _ = SETS[name]
    rng = np.random.default_rng(n + len(v))
    fields = (1 + 0.02 * rng.uniform(-1, 1, n), 0.03 * rng.uniform(-1, 1, n), None,
              th * (1 + 0.02 * rng.uniform(-1, 1, n)))
    lat = _gpu(name, 1, n, 1, 1.3).init(*fields)
    lat.step(25)
    got = [t.cpu().numpy() for t in lat.moments() if t is not None]
    ref = _ref(name, 1, n, 1, 1.3)
    want = ref.moments(ref.step(ref.init(*fields), 25))
    assert rel_err(got[0], want[0]) < 1e-12
    assert rel_err(got[1], want[1], 0.03) < 1e-12
    assert rel_err(got[2], want[3]) < 1e-12


def test_d1q4_shock_tube_matches_oracle():
    """The four-velocity isothermal model (theta0 = 4/3) on the ratio-1.1
    tube of Sec. 3.2, 300 steps with zero-gradient ends."""
    th = 4.0 / 3.0
    fields = inputs.shock_tube(1000, rho_l=1.1, theta_l=th, rho_r=1.0, theta_r=th)
    lat = _gpu("d1q4", 1, 1000, 1, 1.0).init(*fields)
    lat.step(300)
    got = [t.cpu().numpy() for t in lat.moments() if t is not None]
    ref = _ref("d1q4", 1, 1000, 1, 1.0)
    want = ref.moments(ref.step(ref.init(*fields), 300))
    assert rel_err(got[0], want[0]) < 1e-12 and rel_err(got[1], want[1], 0.05) < 1e-12


@pytest.mark.parametrize("name", ["d1q4", "q7"])
def test_step2d_f32_matches_oracle(name):
    v, th, _ = SETS[name]
    steps = 20
    fields = _fields2(300, 40, th, seed=3)
    lat = _gpu(name, 2, 300, 40, 1.6, storage="f32").init(*fields)
    lat.step(steps)
    got = [t.cpu().numpy() for t in lat.moments()]
    ref = _ref(name, 2, 300, 40, 1.6)
    want = ref.moments(ref.step(ref.init(*fields), steps))
    errs = (rel_err(got[0], want[0]), rel_err(got[1], want[1], 0.03),
            rel_err(got[2], want[2], 0.03), rel_err(got[3], want[3]))
    assert max(errs) < steps * 400 * EPS32, errs


@pytest.mark.parametrize("name", sorted(SETS))
def test_sums_conserve(name):
    """Mass and momentum always; the energy sum for the thermal sets."""
    v, th, iso = SETS[name]
    fields = _fields2(64, 48, th, seed=9)
    lat = _gpu(name, 2, 64, 48, 1.5).init(*fields)
    s0 = np.array(lat.sums())
    s1 = np.array(lat.step(30, sums=True))
    assert abs(s1[0] - s0[0]) < 1e-12 * s0[0]
    assert np.abs(s1[1:3] - s0[1:3]).max() < 1e-12 * s0[0]
    if not iso:
        assert abs(s1[3] - s0[3]) < 1e-12 * s0[3]


def test_split_calls_are_bitwise_equal():
    fields = _fields2(300, 20, 1.0, seed=4)
    a = _gpu("q7", 2, 300, 20, 1.5).init(*fields)
    b = _gpu("q7", 2, 300, 20, 1.5).init(*fields)
    a.step(5)
    b.step(2)
    b.step(3)
    assert torch.equal(a.f, b.f)


@pytest.mark.parametrize("name,storage", [("q7", "f32"), ("d1q4", "f32"), ("q7", "f64")])
def test_full_size_sampled_nodes(name, storage):
    """At the 4096^2 KH workload, sampled nodes of one fused step equal the
    oracle's collision of the same pulled populations."""
    v, th, iso = SETS[name]
    q, n = len(v), 4096
    lat = _gpu(name, 2, n, n, 1.8, storage=storage)
    lat.init(*inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80, theta=th))
    lat.step(3)
    before = lat.f.clone()
    lat.step(1)
    after = lat.f
    rng = np.random.default_rng(2)
    ys = np.concatenate([rng.integers(0, n, 30), [0, n - 1, 2]])
    xs = np.concatenate([rng.integers(0, n, 30), [n - 1, 0, 256]])
    k = np.arange(q * q)
    vi, vj = np.array(v)[k % q], np.array(v)[k // q]
    one = oracle.Lattice(2, 1, 1, v=v, omega=1.8, theta0=th if iso else None)
    tol = 1e-14 if storage == "f64" else 64 * EPS32
    for y, x in zip(ys, xs):
        src = (((y - vj) % n) * (q * q) + k) * n + (x - vi) % n
        dst = (y * (q * q) + k) * n + x
        pre = before[torch.from_numpy(src).to(before.device)].double().cpu().numpy()
        got = after[torch.from_numpy(dst).to(after.device)].double().cpu().numpy()
        post = one.step(pre.reshape(q * q, 1, 1), 1).ravel()
        assert np.abs(got - post).max() < tol * np.abs(post).max(), (y, x)
