"""Pins of the oracle's three-dimensional model, the tensor product D3Q125 of
the five-velocity rule over three axes (Sec. 2.4)."""
import numpy as np
import pytest

import oracle


def _fields(shape, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    return (1 + amp * rng.standard_normal(shape), amp * rng.standard_normal(shape),
            amp * rng.standard_normal(shape), amp * rng.standard_normal(shape),
            0.35 + 0.2 * amp * rng.standard_normal(shape))


def test_conservation_periodic():
    lat = oracle.Lattice3(6, 5, 4, omega=1.6)
    f = lat.init(*_fields((4, 5, 6), 1))
    s0 = lat.sums(f)
    s1 = lat.sums(lat.step(f, 20))
    assert abs(s1[0] - s0[0]) < 1e-12 * s0[0]
    assert np.abs(s1[1:4] - s0[1:4]).max() < 1e-12 * s0[0]
    assert abs(s1[4] - s0[4]) < 1e-12 * s0[4]


def test_equilibrium_moments_and_energy():
    """The moments of the tensor-product equilibrium are those of the fields
    (exact to fourth order per axis), so 3 rho theta = sum f |v - u|^2 and
    sum f |v|^2 = rho (3 theta + |u|^2)."""
    fl = _fields((3, 4, 5), 2)
    lat = oracle.Lattice3(5, 4, 3)
    f = lat.init(*fl)
    got = lat.moments(f)
    for a, b in zip(got, fl):
        assert np.abs(a - b).max() < 1e-14
    v = lat.v
    q1d = lat.q1d
    vv = np.array([v[k % q1d] ** 2 + v[(k // q1d) % q1d] ** 2 + v[k // q1d ** 2] ** 2
                   for k in range(lat.q)])
    e = np.tensordot(vv, f, axes=1)
    rho, ux, uy, uz, th = fl
    assert np.abs(e - rho * (3 * th + ux * ux + uy * uy + uz * uz)).max() < 1e-13


def test_uniform_flow_is_a_fixed_point():
    """Exactly a fixed point in exact arithmetic; in FP64 the equilibrium's
    moment round trip moves each population by a few ulps per step (the
    systematic drift of the rounded coefficient table)."""
    lat = oracle.Lattice3(4, 4, 4, omega=1.3)
    one = np.ones((4, 4, 4))
    f = lat.init(one, 0.05 * one, -0.02 * one, 0.03 * one, 0.4 * one)
    steps = 5
    assert np.abs(lat.step(f, steps) - f).max() < steps * 2e-14 * np.abs(f).max()


def test_axis_permutation_symmetry():
    """Exchanging x and z in the fields (and u_x with u_z) exchanges them in
    the result."""
    rho, ux, uy, uz, th = _fields((4, 5, 6), 3)
    a = oracle.Lattice3(6, 5, 4, omega=1.7)
    fa = a.step(a.init(rho, ux, uy, uz, th), 6)
    ma = a.moments(fa)
    t = lambda x: np.transpose(x, (2, 1, 0))
    b = oracle.Lattice3(4, 5, 6, omega=1.7)
    fb = b.step(b.init(t(rho), t(uz), t(uy), t(ux), t(th)), 6)
    mb = b.moments(fb)
    assert np.abs(t(mb[0]) - ma[0]).max() < 1e-14
    assert np.abs(t(mb[1]) - ma[3]).max() < 1e-14 and np.abs(t(mb[3]) - ma[1]).max() < 1e-14
    assert np.abs(t(mb[4]) - ma[4]).max() < 1e-14


def test_shear_wave_viscosity():
    """u_x = U sin(2 pi z / L) decays as exp(-nu k^2 t), nu = (1/omega - 1/2) theta
    (Sec. 2.1 with dt = 1), for the three-dimensional model as in two."""
    L, U, th, steps = 32, 1e-4, 0.35, 150
    z = np.arange(L)[:, None, None] * np.ones((L, 2, 2))
    s = np.sin(2 * np.pi * np.arange(L) / L)
    for omega, tol in ((1.0, 2e-3), (1.6, 2e-2)):
        lat = oracle.Lattice3(2, 2, L, omega=omega)
        one = np.ones((L, 2, 2))
        f = lat.init(one, U * np.sin(2 * np.pi * z / L), 0 * one, 0 * one, th * one)
        amp = lambda g: (lat.moments(g)[1].mean(axis=(1, 2)) * s).sum() / (s * s).sum()
        a0, a1 = amp(f), amp(lat.step(f, steps))
        k = 2 * np.pi / L
        nu = -np.log(a1 / a0) / (k * k * steps)
        assert abs(nu / ((1 / omega - 0.5) * th) - 1) < tol


def test_sound_speed_is_that_of_a_monatomic_gas():
    """A small density wave rho = 1 + eps cos(k z) at rest and uniform theta
    splits into a standing sound wave and an isobaric entropy mode; the
    pressure p = rho theta carries only the sound wave, which oscillates at
    c_s k with c_s^2 = gamma theta, gamma = (D + 2)/D = 5/3 in three
    dimensions: its first zero crossing is at t = pi / (2 c_s k)."""
    L, eps, th = 64, 1e-5, 0.35
    z = np.arange(L)[:, None, None] * np.ones((L, 1, 1))
    c = np.cos(2 * np.pi * np.arange(L) / L)
    lat = oracle.Lattice3(1, 1, L, omega=1.0)
    one = np.ones((L, 1, 1))
    f = lat.init(1 + eps * np.cos(2 * np.pi * z / L), 0 * one, 0 * one, 0 * one, th * one)
    amps = []
    for _ in range(40):
        m = lat.moments(f)
        p = (m[0] * m[4])[:, 0, 0] - th
        amps.append((p * c).sum() / (c * c).sum())
        f = lat.step(f, 1)
    amps = np.array(amps)
    i = int(np.where(amps < 0)[0][0])
    t0 = i - 1 + amps[i - 1] / (amps[i - 1] - amps[i])
    k = 2 * np.pi / L
    cs = np.sqrt(5.0 / 3.0 * th)
    assert abs(t0 / (np.pi / (2 * cs * k)) - 1) < 0.02


def test_sums3_closed_form_on_equilibria():
    """ref_sums3 against closed forms: on the equilibrium of random fields the
    five-velocity rule reproduces the Maxwell moments to fourth order per axis,
    so summed over the box
        sum f = sum rho,  sum f v_a = sum rho u_a  (a = x, y, z),
        sum f |v|^2 = sum rho (3 theta + |u|^2).
    Independent, non-symmetric fields per axis make an exchanged weight (say
    v_y for v_z) or a dropped term fail."""
    shape = (4, 5, 6)
    rho, ux, uy, uz, th = _fields(shape, 7, amp=0.08)
    uy = uy + 0.03            # distinct mean momentum along each axis
    uz = uz - 0.05
    lat = oracle.Lattice3(6, 5, 4, omega=1.3)
    s = lat.sums(lat.init(rho, ux, uy, uz, th))
    ref = np.array([rho.sum(), (rho * ux).sum(), (rho * uy).sum(), (rho * uz).sum(),
                    (rho * (3 * th + ux ** 2 + uy ** 2 + uz ** 2)).sum()])
    assert np.abs(s - ref).max() < 1e-13 * np.abs(ref).max(), (s, ref)
    # the momenta along the three axes differ, so an axis mix-up cannot pass
    assert min(abs(ref[1] - ref[2]), abs(ref[2] - ref[3]), abs(ref[1] - ref[3])) > 0.1
