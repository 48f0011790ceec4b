"""Degenerate cases of the step on the GPU: the rest state, the relaxation
constant at the edge of its range, and calls that do nothing."""
import numpy as np
import pytest
import torch

import oracle
from helpers import pulled_state, rel_err
from paper_1402_5487_amd import inputs
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu


def _rest(nx, ny, th):
    ones = np.ones((ny, nx))
    return ones, 0 * ones, 0 * ones, th * ones


def test_rest_state_is_a_fixed_point_f64():
    """f = rho0 w (u = 0) is an equilibrium: 100 steps change it by rounding only."""
    lat = Lattice(2, 64, 48, omega=1.8).init(*_rest(64, 48, 0.35))
    f0 = pulled_state(lat.f, lat)
    lat.step(100)
    assert np.abs(pulled_state(lat.f, lat) - f0).max() < 1e-15


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_rest_state_stays_at_rest_in_16_bit_storage(storage):
    """At the deviation base the stored deviations start at zero; the FP32
    collision of the rest state reproduces it up to FP32 rounding, so 50
    steps leave rho, u and theta at rest to 1e-6 (the planes' scale is the
    floor 2^-26 rho0 of a zero deviation, so the deviations hold FP32
    rounding noise, not drift)."""
    th = 0.35
    lat = Lattice(2, 300, 20, omega=1.8, storage=storage, theta0=th).init(*_rest(300, 20, th))
    assert int((lat.f.view(torch.int16) & 0x7fff).count_nonzero()) == 0
    lat.step(50)
    rho, ux, uy, tt = (t.cpu().numpy() for t in lat.moments())
    assert np.abs(rho - 1).max() < 1e-6 and np.abs(tt - th).max() < 1e-6
    assert max(np.abs(ux).max(), np.abs(uy).max()) < 1e-6


@pytest.mark.parametrize("omega", [0.05, 1.0, 1.999])
def test_relaxation_constant_range_matches_oracle(omega):
    """Heavy damping, full relaxation and the edge of the stable range."""
    nx, ny, steps = 70, 33, 12
    fields = inputs.random_fields(nx, ny, seed=int(omega * 1000), u=0.02)
    lat = Lattice(2, nx, ny, omega=omega).init(*fields)
    lat.step(steps)
    ref = oracle.Lattice(2, nx, ny, omega=omega)
    f = ref.step(ref.init(*fields), steps)
    assert rel_err(pulled_state(lat.f, lat), f) < 1e-12


def test_zero_steps_change_nothing():
    fields = inputs.random_fields(40, 12, seed=4)
    lat = Lattice(2, 40, 12, omega=1.5).init(*fields)
    before = lat.f.clone()
    s = lat.step(0, sums=True)
    assert torch.equal(lat.f, before) and lat.cur == 0
    assert abs(s[0] - pulled_state(before, lat).sum()) < 1e-12 * s[0]
