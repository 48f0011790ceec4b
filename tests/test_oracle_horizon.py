"""The oracle's own rounding-order floor (its self-divergence).

Beyond the parity horizon no two correct FP64 implementations agree to 1e-12:
ulp-level differences in operation order grow with the flow's instabilities
(the shear layers of the Kelvin-Helmholtz problem).  The oracle can sum each
node's populations in reversed order (`reverse_sums=True`), an equally
correct rounding of the same discrete moments, and the distance between the
two runs is the floor that a GPU run past the horizon is compared with.

These tests pin that mode on the 256^2 KH problem (theta = 0.35 stable
variant, omega = 1.8, delta = L/80):
  * after one step the two runs differ, and only at the level of rounding
    (the reordered 25-term sums);
  * both conserve mass and energy to FP64 rounding (Eq. srt conserves them
    exactly in rationals);
  * within 500 steps the divergence stays below the 1e-12 parity bound,
    which is the horizon the 256^2 parity claims rely on.
"""
import numpy as np
import pytest

import oracle
from paper_1402_5487_amd import inputs

N, OMEGA, THETA = 256, 1.8, 0.35


def _fields_rel(a, b, u0=0.1):
    return max(float(np.abs(x - y).max() / max(np.abs(y).max(), fl))
               for x, y, fl in zip(a, b, (1.0, u0, u0, 1.0)))


@pytest.fixture(scope="module")
def runs():
    lat = oracle.Lattice(2, N, N, omega=OMEGA)
    f0 = lat.init(*inputs.kelvin_helmholtz(N, N, u0=0.1, delta=N / 80.0, theta=THETA))
    a, b = f0, f0
    out = {"sums0": lat.sums(f0)}
    for t in (1, 100, 500):
        n = t - out.get("t", 0)
        a = lat.step(a, n)
        b = lat.step(b, n, reverse_sums=True)
        out["t"] = t
        out[t] = (_fields_rel(lat.moments(b, reverse_sums=True), lat.moments(a)),
                  lat.sums(a), lat.sums(b))
    return out


def test_reversed_order_changes_only_the_rounding(runs):
    # a reordered sum of 25 FP64 terms moves by at most ~25 ulps of the sum
    # of their magnitudes; the temperature's terms f |v - u|^2 reach 18 f, so
    # relative field differences of a few 1e-15 are rounding, 1e-14 is not
    d1 = runs[1][0]
    assert 0.0 < d1 < 1e-14, d1


def test_both_orders_conserve(runs):
    s0 = runs["sums0"]
    for t in (100, 500):
        for s in runs[t][1:]:
            assert abs(s[0] / s0[0] - 1) < 1e-13 and abs(s[3] / s0[3] - 1) < 1e-13
            assert max(abs(s[1] - s0[1]), abs(s[2] - s0[2])) < 1e-13 * s0[0]


def test_self_divergence_inside_the_horizon(runs):
    d100, d500 = runs[100][0], runs[500][0]
    print(f"oracle self-divergence 256^2 KH: step 1 {runs[1][0]:.2e}, "
          f"100 {d100:.2e}, 500 {d500:.2e}", flush=True)
    assert d500 < 1e-12, d500
