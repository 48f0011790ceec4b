"""Seeded synthetic initial fields for the test problems of arXiv:1402.5487.

This module only draws and lays out initial macroscopic fields (rho, u, theta)
and run parameters; it holds none of the method's arithmetic, so both the GPU
library's tests and the CPU oracle consume the same inputs.  All arrays are
float64 with shape (ny, nx) in 2D and (nx,) in 1D; node (i, j) sits at x = i,
y = j in lattice units.
"""
from dataclasses import dataclass

import numpy as np


def kelvin_helmholtz(nx, ny=None, u0=0.1, delta=None, theta=0.35, uy_amp=0.005,
                     rho=1.0, mode=1, phase=0.0):
    """Double shear layer (Sec. 3.2 and Sec. 4 of the paper), in lattice units.

    u_x = u0 tanh((y - L/4)/delta) for y < L/2, u0 tanh((3L/4 - y)/delta)
    otherwise (L = ny, delta = L/80 by default); u_y = uy_amp sin(2 pi m x / nx
    + phase); uniform rho and theta.  The paper's x + 1/4 phase and relative
    amplitude are replaced by an absolute amplitude and an explicit phase.
    """
    ny = nx if ny is None else ny
    L = float(ny)
    delta = L / 80.0 if delta is None else float(delta)
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    ux_col = np.where(y < L / 2, u0 * np.tanh((y - L / 4) / delta),
                      u0 * np.tanh((3 * L / 4 - y) / delta))
    ux = np.broadcast_to(ux_col, (ny, nx)).copy()
    uy = np.broadcast_to(uy_amp * np.sin(2 * np.pi * mode * x / nx + phase),
                         (ny, nx)).copy()
    return (np.full((ny, nx), rho), ux, uy, np.full((ny, nx), theta))


def shock_tube(n=1000, rho_l=1.0, theta_l=0.5, rho_r=0.125, theta_r=0.4):
    """1D Riemann problem: nodes [0, n/2) hold the left state, the rest the
    right state, u = 0 everywhere."""
    x = np.arange(n)
    left = x < n // 2
    rho = np.where(left, rho_l, rho_r).astype(np.float64)
    theta = np.where(left, theta_l, theta_r).astype(np.float64)
    return rho, np.zeros(n), None, theta


def shear_wave(nx, ny=None, amp=1e-4, theta=0.35, rho=1.0, along="x"):
    """Decaying transverse wave u_x = amp sin(2 pi y / ny) (or the transposed
    wave u_y = amp sin(2 pi x / nx))."""
    ny = nx if ny is None else ny
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    x = np.arange(nx, dtype=np.float64)[None, :] * np.ones((ny, 1))
    z = np.zeros((ny, nx))
    if along == "x":
        ux, uy = amp * np.sin(2 * np.pi * y / ny), z.copy()
    else:
        ux, uy = z.copy(), amp * np.sin(2 * np.pi * x / nx)
    return np.full((ny, nx), rho), ux, uy, np.full((ny, nx), theta)


def random_fields(nx, ny, seed, theta=(0.34, 0.36), u=0.05, drho=0.02):
    """Smooth-free random fields near a rest state (used to exercise every
    node independently in parity tests)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + drho * rng.uniform(-1, 1, (ny, nx))
    ux = u * rng.uniform(-1, 1, (ny, nx))
    uy = u * rng.uniform(-1, 1, (ny, nx))
    th = rng.uniform(theta[0], theta[1], (ny, nx))
    return rho, ux, uy, th


def random_fields_3d(nx, ny, nz, seed, theta=(0.34, 0.36), u=0.05, drho=0.02):
    """random_fields on an (nz, ny, nx) lattice: (rho, ux, uy, uz, theta)."""
    rng = np.random.default_rng(seed)
    shp = (nz, ny, nx)
    rho = 1.0 + drho * rng.uniform(-1, 1, shp)
    ux, uy, uz = (u * rng.uniform(-1, 1, shp) for _ in range(3))
    th = rng.uniform(theta[0], theta[1], shp)
    return rho, ux, uy, uz, th


def taylor_green_3d(nx, ny=None, nz=None, u0=0.05, theta=1.0 / 3.0, rho=1.0):
    """Three-dimensional Taylor-Green vortex on an (nz, ny, nx) periodic box:
    u = u0 (sin X cos Y cos Z, -cos X sin Y cos Z, 0) with X = 2 pi x / nx
    etc., uniform density and temperature (the classic decaying-vortex test
    of three-dimensional solvers)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    X = 2 * np.pi * np.arange(nx) / nx
    Y = 2 * np.pi * np.arange(ny) / ny
    Z = 2 * np.pi * np.arange(nz) / nz
    Zg, Yg, Xg = np.meshgrid(Z, Y, X, indexing="ij")
    ux = u0 * np.sin(Xg) * np.cos(Yg) * np.cos(Zg)
    uy = -u0 * np.cos(Xg) * np.sin(Yg) * np.cos(Zg)
    uz = np.zeros_like(ux)
    shp = ux.shape
    return np.full(shp, rho), ux, uy, uz, np.full(shp, theta)


@dataclass
class BatchMember:
    side: int
    u0: float
    theta: float
    omega: float


def batch_members(count=256, seed=0, sides=tuple(range(64, 513, 32)),
                  theta_range=(0.2, 0.4), omega_range=(1.5, 1.9),
                  u0_range=(0.02, 0.12)):
    """Independent KH lattices for the batching form: per lattice the draws
    are made in the order (side, U0, theta, omega) from one generator."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        side = int(sides[rng.integers(0, len(sides))])
        u0 = float(rng.uniform(*u0_range))
        th = float(rng.uniform(*theta_range))
        om = float(rng.uniform(*omega_range))
        out.append(BatchMember(side, u0, th, om))
    return out


@dataclass
class ClosureSeed:
    seed: int
    u0: float
    uy_amp: float
    mode: int
    phase: float


def closure_seed(seed):
    """KH variations used to train and judge the learned closure."""
    rng = np.random.default_rng(seed)
    return ClosureSeed(seed, float(rng.uniform(0.04, 0.12)),
                       float(rng.uniform(0.003, 0.008)),
                       int(rng.integers(1, 3)), float(rng.uniform(0, 2 * np.pi)))
