"""GPU parity: the HIP library against the FP64 oracle on identical seeded
inputs, through the C ABI.

Tolerances
  * FP64 storage: 1e-12 relative (fields normalised by max(|ref|, 1); the
    velocity by max(|u_ref|, U0)), inside the parity horizon of each case
    (stable S-variant parameters, or few steps for the unstable literal ones).
  * FP32 storage: each step rounds every population once on store and runs
    ~10 dependent FP32 operations on it, so a field built from 25 populations
    moves by at most ~25 * 8 eps32 per step relative to its scale; the bound
    used is n_steps * 200 * eps32.
  * 16-bit deviation storage: a stored deviation |h| <= 2^10 (the scale rule)
    rounds by at most half an ulp of the top binade: 2^-2 (FP16) or 2 (BF16)
    times the plane's scale.  The bound used is n_steps * sum_k of that.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import rest_weights, V5, pulled_state, rel_err
from paper_1402_5487_amd import _plbm, inputs
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

EPS32 = np.finfo(np.float32).eps


def _run_both(nx, ny, fields, omega, steps, storage="f64", theta0=None, rounding="nearest"):
    lat = Lattice(2, nx, ny, omega=omega, storage=storage, theta0=theta0, rounding=rounding)
    lat.init(*fields)
    lat.step(steps)
    got = [t.cpu().numpy() for t in lat.moments()]
    ref_lat = oracle.Lattice(2, nx, ny, omega=omega)
    f = ref_lat.step(ref_lat.init(*fields), steps)
    ref = ref_lat.moments(f)
    return lat, got, ref, f


def _field_errs(got, ref, u0):
    return (rel_err(got[0], ref[0]), rel_err(got[1], ref[1], u0),
            rel_err(got[2], ref[2], u0), rel_err(got[3], ref[3]))


# --------------------------------------------------------------------------
# initialisation and moments
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny", [(3, 3), (7, 4), (300, 37)])
def test_init_then_moments_is_identity(nx, ny):
    fields = inputs.random_fields(nx, ny, seed=nx, theta=(0.3, 0.6), u=0.2)
    lat = Lattice(2, nx, ny, omega=1.5).init(*fields)
    got = [t.cpu().numpy() for t in lat.moments()]
    for a, b in zip(got, fields):
        assert np.abs(a - b).max() < 4e-15


def test_init_populations_match_oracle():
    fields = inputs.random_fields(41, 23, seed=1)
    lat = Lattice(2, 41, 23, omega=1.5).init(*fields)
    ref = oracle.Lattice(2, 41, 23, omega=1.5).init(*fields)
    # different but equally valid rounding order (moment recurrence, FMA)
    assert np.abs(pulled_state(lat.f, lat) - ref).max() < 2e-15 * np.abs(ref).max()


# --------------------------------------------------------------------------
# FP64 step parity (several tiles in x and y, ragged tails, wrap seams)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,steps", [(3, 3, 20), (7, 5, 30), (300, 37, 40),
                                         (800, 45, 25), (513, 19, 33)])
def test_step_f64_random_fields(nx, ny, steps):
    fields = inputs.random_fields(nx, ny, seed=nx * 7 + ny)
    lat, got, ref, f = _run_both(nx, ny, fields, 1.7, steps)
    assert max(_field_errs(got, ref, 0.05)) < 1e-12
    assert rel_err(pulled_state(lat.f, lat), f) < 1e-12


def test_step_f64_kelvin_helmholtz_stable_variant():
    fields = inputs.kelvin_helmholtz(300, 128, u0=0.1, theta=0.35)
    lat, got, ref, _ = _run_both(300, 128, fields, 1.8, 200)
    assert max(_field_errs(got, ref, 0.1)) < 1e-12


def _floor_run(n, theta, checkpoints):
    """GPU FP64 run, oracle run and the oracle with reversed per-node
    summation (its self-divergence) on the KH problem at n^2, compared at
    each checkpoint: (step, GPU vs oracle, oracle vs reversed oracle)."""
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80, theta=theta)
    lat = Lattice(2, n, n, omega=1.8, storage="f64").init(*fields)
    ref_lat = oracle.Lattice(2, n, n, omega=1.8)
    a = b = ref_lat.init(*fields)
    out, t = [], 0
    for c in checkpoints:
        lat.step(c - t)
        a = ref_lat.step(a, c - t)
        b = ref_lat.step(b, c - t, reverse_sums=True)
        t = c
        ref = ref_lat.moments(a)
        gpu = max(_field_errs([x.cpu().numpy() for x in lat.moments()], ref, 0.1))
        floor = max(_field_errs(ref_lat.moments(b, reverse_sums=True), ref, 0.1))
        print(f"KH {n}^2 theta={theta} step {c}: GPU vs oracle {gpu:.3e}, "
              f"oracle self-divergence {floor:.3e}", flush=True)
        out.append((c, gpu, floor))
    return out


@pytest.mark.timeout(900)
def test_step_f64_kelvin_helmholtz_1024_horizon():
    """The 1024^2 KH configuration (delta = L/80 = 12.8, theta = 0.35,
    omega = 1.8) in FP64 against the oracle for the whole 2000-step parity
    horizon (about two minutes of oracle time): 1e-12 at every checkpoint,
    and never more than 10x the oracle's own rounding-order floor (its
    distance to the same oracle with reversed per-node summation; measured
    ratio 2-3.3)."""
    for step, gpu, floor in _floor_run(1024, 0.35, (500, 1000, 2000)):
        assert gpu < 1e-12, (step, gpu)
        assert gpu <= 10 * floor, (step, gpu, floor)


def test_step_f64_past_the_horizon_within_the_oracle_floor():
    """Past the parity horizon: the literal theta = 0.3 state grows round-off
    by about 8 % per step, so by step 400 two correct FP64 runs differ at
    the 1e-2 level.  There the GPU's distance to the oracle must stay within
    10x of the oracle's distance to itself under reversed summation
    (measured ratio 0.8-1.2 from 4e-14 to 1e-2)."""
    rows = _floor_run(256, 0.3, (100, 200, 300, 400))
    for step, gpu, floor in rows:
        assert gpu <= 10 * floor, (step, gpu, floor)
    assert rows[-1][2] > 1e-6          # genuinely past the 1e-12 horizon


def test_step_f64_kelvin_helmholtz_literal_within_horizon():
    """theta = 0.3 is linearly unstable (growth ~1.06 per step); 60 steps keep
    rounding differences ~1e-15 x 1.06^60 far below the bound."""
    fields = inputs.kelvin_helmholtz(260, 64, u0=0.1, theta=0.3)
    _, got, ref, _ = _run_both(260, 64, fields, 1.8, 60)
    assert max(_field_errs(got, ref, 0.1)) < 1e-12


@pytest.mark.parametrize("storage,rounding", [("f64", "nearest"), ("f16dev", "stochastic"),
                                              ("bf16dev", "stochastic")])
def test_split_calls_are_bitwise_equal(storage, rounding):
    """Deterministic whatever the split of the steps into calls; for
    stochastic rounding too, since its random bits hash the node, the
    population and the value."""
    fields = inputs.random_fields(270, 20, seed=3)
    kw = dict(omega=1.6, storage=storage, rounding=rounding,
              theta0=0.35 if storage != "f64" else None)
    a = Lattice(2, 270, 20, **kw).init(*fields)
    b = Lattice(2, 270, 20, **kw).init(*fields)
    a.step(9)
    for _ in range(9):
        b.step(1)
    assert torch.equal(a.f, b.f)
    c = Lattice(2, 270, 20, **kw).init(*fields)
    c.step(9)
    assert torch.equal(a.f, c.f)


# --------------------------------------------------------------------------
# FP32 storage and 16-bit deviation storage against the FP64 oracle
# --------------------------------------------------------------------------

def test_step_f32_parity():
    steps = 40
    fields = inputs.kelvin_helmholtz(300, 40, u0=0.1, theta=0.35)
    _, got, ref, _ = _run_both(300, 40, fields, 1.8, steps, storage="f32")
    errs = _field_errs(got, ref, 0.1)
    assert max(errs) < steps * 200 * EPS32, errs


@pytest.mark.parametrize("rounding", ["nearest", "stochastic"])
@pytest.mark.parametrize("storage,half_ulp", [("f16dev", 2.0 ** -2), ("bf16dev", 2.0)])
def test_step_dev_storage_parity(storage, half_ulp, rounding):
    steps = 40
    th = 0.35
    fields = inputs.kelvin_helmholtz(300, 40, u0=0.1, theta=th)
    lat, got, ref, _ = _run_both(300, 40, fields, 1.8, steps, storage=storage, theta0=th,
                                 rounding=rounding)
    # one store rounds by at most half an ulp (nearest) or one ulp (stochastic)
    ulps = 1.0 if rounding == "nearest" else 2.0
    per_store = ulps * half_ulp * sum(lat.desc.scale[k] for k in range(25))
    bound = steps * per_store
    errs = _field_errs(got, ref, 1.0)
    assert errs[0] < bound and errs[3] < bound / 0.35, (errs, bound)
    assert errs[1] < 3 * bound and errs[2] < 3 * bound, (errs, bound)


@pytest.mark.parametrize("nx", [512, 300])     # whole 256-node tiles, and a ragged last tile
def test_f32_step_matches_oracle_step_per_population(nx):
    """One FP32 step from the GPU's own FP32 state, population by population,
    against the oracle's FP64 step of the same state.  The FP32 collision
    rounds the moments relative to the node's mass, and those errors of a few
    eps32 rho reach every population through its sensitivity to u and theta:
    the +-3 planes hold 1e-4 to 1e-8 of rho yet carry errors of up to a few
    eps32 rho (a float32 emulation of the kernel's operation order gives at
    most 3.6 eps32 rho).  The bound is 64 eps32 relative plus 8 eps32 rho
    absolute; the large populations, which it bounds relatively, sit at
    about a tenth of it."""
    ny, th = 24, 0.35
    fields = inputs.kelvin_helmholtz(nx, ny, u0=0.1, delta=3.0, theta=th)
    lat = Lattice(2, nx, ny, omega=1.8, storage="f32").init(*fields)
    lat.step(3)
    pre = pulled_state(lat.f, lat)
    lat.step(1)
    got = pulled_state(lat.f, lat)
    ref = oracle.Lattice(2, nx, ny, omega=1.8).step(pre, 1)
    rho = pre.sum(axis=0).max()
    bound = 64 * EPS32 * np.abs(ref) + 8 * EPS32 * rho
    ratio = np.abs(got - ref) / bound
    big = np.abs(ref) > 0.01 * rho
    print(f"f32 per-population error / bound: max {ratio.max():.3f}, "
          f"largest populations {ratio[big].max():.3f}", flush=True)
    assert np.all(ratio <= 1.0), float(ratio.max())


@pytest.mark.parametrize("rounding", ["nearest", "stochastic"])
@pytest.mark.parametrize("storage,half_ulp", [("f16dev", 2.0 ** -2), ("bf16dev", 2.0)])
@pytest.mark.parametrize("nx", [512, 300])     # whole 256-node tiles, and a ragged last tile
def test_dev_storage_step_matches_oracle_step(storage, half_ulp, nx, rounding):
    """One step from the GPU's own 16-bit state, population by population:
    the oracle's FP64 step of the decoded state, within the rounding of the
    stored deviation (half an ulp of |h| < 2^10 for nearest, doubled for
    growth, which also covers the one ulp of stochastic rounding) plus FP32
    arithmetic."""
    ny, th = 24, 0.35
    fields = inputs.kelvin_helmholtz(nx, ny, u0=0.1, delta=3.0, theta=th)
    lat = Lattice(2, nx, ny, omega=1.8, storage=storage, theta0=th,
                  rounding=rounding).init(*fields)
    lat.step(3)
    pre = pulled_state(lat.f, lat)
    lat.step(1)
    got = pulled_state(lat.f, lat)
    ref = oracle.Lattice(2, nx, ny, omega=1.8).step(pre, 1)
    scale = np.array([lat.desc.scale[k] for k in range(25)])
    # population k of the pulled state was stored with the scale of k
    bound = 2 * half_ulp * scale[:, None, None] + 64 * EPS32 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound), float((np.abs(got - ref) / bound).max())


# --------------------------------------------------------------------------
# 1D D1Q5 shock tube with zero-gradient ghost ends
# --------------------------------------------------------------------------

def _run_1d(fields, omega, steps, n):
    lat = Lattice(1, n, omega=omega).init(*fields)
    lat.step(steps)
    got = [None if t is None else t.cpu().numpy() for t in lat.moments()]
    ref_lat = oracle.Lattice(1, n, omega=omega, bc=1)
    f = ref_lat.step(ref_lat.init(*fields), steps)
    return lat, got, ref_lat.moments(f), f


def test_shock_tube_stable_variant_500_steps():
    fields = inputs.shock_tube(1000, rho_r=0.5)
    lat, got, ref, f = _run_1d(fields, 1.0, 500, 1000)
    assert rel_err(got[0], ref[0]) < 1e-12
    assert rel_err(got[1], ref[1], 0.1) < 1e-12
    assert rel_err(got[3], ref[3]) < 1e-12
    assert rel_err(pulled_state(lat.f, lat), f) < 1e-12


def test_shock_tube_literal_within_horizon():
    """The literal tube (rho_R = 0.125) is unstable past its rarefaction;
    compare while rounding differences stay small (15 steps)."""
    fields = inputs.shock_tube(1000)
    _, got, ref, _ = _run_1d(fields, 1.0, 15, 1000)
    assert rel_err(got[0], ref[0]) < 1e-12 and rel_err(got[3], ref[3]) < 1e-12


def test_shock_tube_literal_blows_up_and_is_reported():
    lat = Lattice(1, 1000, omega=1.0).init(*inputs.shock_tube(1000))
    with pytest.raises(_plbm.PlbmError) as e:
        lat.step(500, sums=True)
    assert e.value.status == _plbm.PLBM_ENONFINITE


@pytest.mark.parametrize("n", [1, 2, 5, 257])
def test_tiny_and_ragged_1d(n):
    fields = inputs.random_fields(n, 1, seed=n)
    fields = (fields[0][0], fields[1][0], None, fields[3][0])
    _, got, ref, _ = _run_1d(fields, 1.3, 12, n)
    assert rel_err(got[0], ref[0]) < 1e-12 and rel_err(got[1], ref[1], 0.05) < 1e-12


# --------------------------------------------------------------------------
# invariants (fused FP64 sums) and failure reporting
# --------------------------------------------------------------------------

def test_fused_sums_match_oracle_and_conserve():
    fields = inputs.random_fields(600, 50, seed=9)
    lat = Lattice(2, 600, 50, omega=1.8).init(*fields)
    s0 = lat.sums()
    s1 = lat.step(30, sums=True)
    ref_lat = oracle.Lattice(2, 600, 50, omega=1.8)
    ref0 = ref_lat.sums(ref_lat.init(*fields))
    assert abs(s0[0] / ref0[0] - 1) < 1e-14 and abs(s0[3] / ref0[3] - 1) < 1e-14
    assert abs(s1[0] / s0[0] - 1) < 1e-13 and abs(s1[3] / s0[3] - 1) < 1e-13
    assert max(abs(s1[1] - s0[1]), abs(s1[2] - s0[2])) < 1e-13 * s0[0]
    s2 = lat.sums()
    assert abs(s2[0] / s1[0] - 1) < 1e-14


def test_nan_input_reported_as_nonfinite():
    rho, ux, uy, th = inputs.random_fields(40, 30, seed=2)
    rho[5, 7] = np.nan
    lat = Lattice(2, 40, 30, omega=1.5).init(rho, ux, uy, th)
    with pytest.raises(_plbm.PlbmError) as e:
        lat.step(3, sums=True)
    assert e.value.status == _plbm.PLBM_ENONFINITE


def test_checkpoint_resume_is_bitwise():
    fields = inputs.random_fields(280, 24, seed=4)
    a = Lattice(2, 280, 24, omega=1.7).init(*fields)
    a.step(10)
    st = a.state_dict()
    a.step(7)
    b = Lattice(2, 280, 24, omega=1.7)
    b.load_state_dict(st)
    b.step(7)
    assert torch.equal(a.f, b.f)


# --------------------------------------------------------------------------
# the benchmark's full size, sampled: every sampled node's post-collision
# populations equal the oracle's collision of the same pulled state
# --------------------------------------------------------------------------

@pytest.mark.parametrize("storage,rounding", [("f64", "nearest"), ("f32", "nearest"), ("f16dev", "nearest"),
                                              ("bf16dev", "nearest"), ("f16dev", "stochastic"),
                                              ("bf16dev", "stochastic")])
def test_full_size_sampled_nodes(storage, rounding):
    n = 4096
    dev = storage.endswith("dev")
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80, theta=0.35)
    lat = Lattice(2, n, n, omega=1.8, storage=storage, theta0=0.35 if dev else None, rounding=rounding)
    lat.init(*fields)
    lat.step(3)
    before = lat.f.clone()
    lat.step(1)
    after = lat.f
    rng = np.random.default_rng(0)
    ys = np.concatenate([rng.integers(0, n, 40), [0, 1, 2, n - 1, n - 3]])
    xs = np.concatenate([rng.integers(0, n, 40), [n - 1, 0, 255, 256, 3]])
    plane = n * n
    # device layout: (y * 25 + k) * n + x
    src = before.view(n, 25, n).transpose(0, 1)
    dst = after.view(n, 25, n).transpose(0, 1)
    one = oracle.Lattice(2, 1, 1, omega=1.8)
    tol = 1e-14 if storage == "f64" else 64 * EPS32
    if dev:
        w = rest_weights(lat.desc.theta0)
        base = np.array([lat.desc.rho0 * w[k % 5] * w[k // 5] for k in range(25)],
                        dtype=np.float32).astype(np.float64)
        scale = np.array([lat.desc.scale[k] for k in range(25)])
        dec = lambda h, k: base[k] + scale[k] * float(h)
    else:
        dec = lambda h, k: float(h)
    for y, x in zip(ys, xs):
        pre = np.array([dec(src[k, (y - V5[k // 5]) % n, (x - V5[k % 5]) % n].double().item(), k)
                        for k in range(25)]).reshape(25, 1, 1)
        post = one.step(pre, 1).ravel()       # 1x1 periodic lattice: pure collision
        got = np.array([dec(dst[k, y, x].double().item(), k) for k in range(25)])
        if dev:
            # an ulp of the stored deviation (|h| < 2^10: 2^-1 in FP16, 2^2 in
            # BF16), half of it for round to nearest, doubled, plus FP32
            ulp = 2.0 ** -1 if storage == "f16dev" else 2.0 ** 2
            bound = 2 * (ulp / 2 if rounding == "nearest" else ulp) * scale + 64 * EPS32 * np.abs(post)
            assert np.all(np.abs(got - post) <= bound), (y, x)
        else:
            assert np.abs(got - post).max() < tol * np.abs(post).max(), (y, x)
    assert plane == n * n
