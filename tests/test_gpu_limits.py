"""Lattices at the edges of the launch geometry: more rows than a grid's y
dimension holds (65536), and rows as long as the descriptor allows (2^26
nodes, where the 32-bit lane offsets reach their largest values)."""
import numpy as np
import pytest
import torch

import oracle
from helpers import V5, pulled_state, rel_err
from paper_1402_5487_amd import inputs
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

EPS32 = np.finfo(np.float32).eps
TALL = 70000


def _compare(lat, ref, fields, steps, u_floor=0.05):
    lat.step(steps)
    got = [t.cpu().numpy() for t in lat.moments()]
    f = ref.step(ref.init(*fields), steps)
    want = ref.moments(f)
    assert rel_err(got[0], want[0]) < 1e-12
    assert max(rel_err(got[1], want[1], u_floor), rel_err(got[2], want[2], u_floor)) < 1e-12
    return f


def test_tall_d2q25_f64_matches_oracle():
    fields = inputs.random_fields(4, TALL, seed=70)
    lat = Lattice(2, 4, TALL, omega=1.6).init(*fields)
    f = _compare(lat, oracle.Lattice(2, 4, TALL, omega=1.6), fields, 6)
    assert rel_err(pulled_state(lat.f, lat), f) < 1e-12
    s = lat.sums()
    assert abs(s[0] - f.sum()) < 1e-12 * s[0]


def test_tall_d2q25_f16dev_step_matches_oracle_step():
    """dev_scales, init, step and moments on a tall 16-bit lattice: one step
    from the GPU's own state equals the oracle's within the storage bound."""
    nx, th = 4, 0.35
    fields = inputs.kelvin_helmholtz(nx, TALL, u0=0.1, delta=TALL / 80, theta=th)
    lat = Lattice(2, nx, TALL, omega=1.8, storage="f16dev", theta0=th).init(*fields)
    rho = lat.moments()[0].cpu().numpy()
    assert np.abs(rho - fields[0]).max() < 1e-3
    lat.step(2)
    pre = pulled_state(lat.f, lat)
    lat.step(1)
    got = pulled_state(lat.f, lat)
    ref = oracle.Lattice(2, nx, TALL, omega=1.8).step(pre, 1)
    scale = np.array([lat.desc.scale[k] for k in range(25)])
    # half an ulp of a stored FP16 deviation (|h| < 2^10) is 2^-2 scale, doubled
    bound = 2 * 2.0 ** -2 * scale[:, None, None] + 64 * EPS32 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)


def test_tall_d2q9_f64_matches_oracle():
    fields = inputs.random_fields(5, TALL, seed=71, theta=(0.25, 0.25))
    lat = Lattice(2, 5, TALL, omega=1.7, zeta=4.0).init(*fields)
    _compare(lat, oracle.Lattice(2, 5, TALL, v=[0, 1, -1], omega=1.7, theta0=0.25), fields, 6)


def test_tall_general_set_f64_matches_oracle():
    v, th = (1, -1, 3, -3), 4.0 / 3.0
    fields = inputs.random_fields(3, TALL, seed=72, theta=(th, th))
    lat = Lattice(2, 3, TALL, omega=1.5, velocities=v, theta0=th).init(*fields)
    _compare(lat, oracle.Lattice(2, 3, TALL, v=list(v), omega=1.5, theta0=th), fields, 6)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_longest_rows_sampled_nodes(storage):
    """nx = 2^26 (the longest row the descriptor accepts), ny = 3: sampled
    nodes of one fused step, at both seams and far along the row, equal the
    oracle's collision of the same pulled populations."""
    nx, ny = 1 << 26, 3
    x = np.arange(nx)
    ux = np.broadcast_to(0.05 * np.sin(2 * np.pi * x / nx * 64), (ny, nx))
    uy = np.broadcast_to(0.02 * np.cos(2 * np.pi * x / nx * 16), (ny, nx))
    rho = np.ones((ny, nx))
    th = np.full((ny, nx), 0.35)
    lat = Lattice(2, nx, ny, omega=1.8, storage=storage)
    lat.init(rho, ux, uy, th)
    del ux, uy, rho, th
    lat.step(2)
    before = lat.f.clone()
    lat.step(1)
    after = lat.f
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.integers(0, nx, 12), [0, 1, 2, nx - 3, nx - 1, nx - 256, (1 << 25) + 7]])
    ys = np.concatenate([rng.integers(0, ny, 12), [0, 2, 1, 0, 2, 1, 1]])
    k = np.arange(25)
    vi, vj = np.array(V5)[k % 5], np.array(V5)[k // 5]
    one = oracle.Lattice(2, 1, 1, omega=1.8)
    tol = 1e-14 if storage == "f64" else 64 * EPS32
    for yy, xx in zip(ys, xs):
        src = (((yy - vj) % ny) * 25 + k) * nx + (xx - vi) % nx
        dst = (yy * 25 + k) * nx + xx
        pre = before[torch.from_numpy(src).to(before.device)].double().cpu().numpy()
        got = after[torch.from_numpy(dst).to(after.device)].double().cpu().numpy()
        post = one.step(pre.reshape(25, 1, 1), 1).ravel()
        assert np.abs(got - post).max() < tol * np.abs(post).max(), (yy, xx)
    del before
    torch.cuda.empty_cache()
