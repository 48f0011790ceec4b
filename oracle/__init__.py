"""FP64 CPU oracle of the parametric lattice Boltzmann method (arXiv:1402.5487).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports it and
shares no code with it.  Every function cites the passage of the paper it
follows; the C core lives in ref_plbm.c.

Array conventions: populations are float64 arrays of shape (q, ny, nx) in 2D
(k = i + q1d * j, i the x velocity index, j the y velocity index) and (q, nx)
in 1D; they hold the pre-collision state f(x, t) of Eq. srt.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    i, d = ctypes.c_int, ctypes.c_double
    lib.ref_lagrange_coeffs.argtypes = [i, _D, _D]
    lib.ref_maxwell_moments.argtypes = [d, d, i, _D]
    lib.ref_maxwell_moments.restype = None
    lib.ref_weights_1d.argtypes = [i, _D, d, d, _D]
    lib.ref_weights_1d.restype = None
    lib.ref_init.argtypes = [i, i, i, i, _D, _D, _D, _D, _D, _D, _D]
    lib.ref_step.argtypes = [i, i, i, i, _D, _D, d, i, _D, i, i]
    lib.ref_step_theta0.argtypes = [i, i, i, i, _D, _D, d, i, d, _D, i, i]
    lib.ref_moments.argtypes = [i, i, i, i, _D, _D, _D, _D, _D, _D, i]
    lib.ref_sums.argtypes = [i, i, i, i, _D, _D, _D]
    lib.ref_num_threads.argtypes = []
    lib.ref_set_num_threads.argtypes = [i]
    lib.ref_set_num_threads.restype = None
    lib.ref_init3.argtypes = [i, i, i, i, _D, _D, _D, _D, _D, _D, _D, _D]
    lib.ref_step3.argtypes = [i, i, i, i, _D, _D, d, _D, i]
    lib.ref_moments3.argtypes = [i, i, i, i, _D, _D, _D, _D, _D, _D, _D]
    lib.ref_sums3.argtypes = [i, i, i, i, _D, _D, _D]
    _lib = lib
    return lib


def num_threads():
    """Threads the oracle's OpenMP loops use."""
    return int(_load().ref_num_threads())


def set_num_threads(n):
    """Threads of the oracle's OpenMP loops from now on (results are the same
    for any count)."""
    _load().ref_set_num_threads(int(n))


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# Paper order of the five thermal velocities (Sec. 2.4: v1 = 0, v2,3 = +-a,
# v4,5 = +-b), with a = 1, b = 3 lattice units.
V_D1Q5 = (0.0, 1.0, -1.0, 3.0, -3.0)


def lagrange_coeffs(v):
    """c[i, j] = coefficient of v^j in the Lagrange polynomial L_i
    (Sec. 2.1, Eq. rdr and the definition of c_ij that follows it)."""
    v = _f64(v)
    q = v.size
    c = np.zeros((q, q))
    rc = _load().ref_lagrange_coeffs(q, _p(v), _p(c))
    if rc != 0:
        raise ValueError("velocity set is invalid (size or duplicates)")
    return c


def maxwell_moments(u, theta, nmax):
    """mu_0..mu_nmax of the 1D Maxwell-Boltzmann distribution (Sec. 2.1)."""
    mu = np.zeros(nmax + 1)
    _load().ref_maxwell_moments(float(u), float(theta), nmax, _p(mu))
    return mu


def weights_1d(c, u, theta):
    """r_i = sum_j c_ij mu_(j-1)(u, theta)  (Eq. rdr)."""
    c = _f64(c)
    q = c.shape[0]
    r = np.zeros(q)
    _load().ref_weights_1d(q, _p(c), float(u), float(theta), _p(r))
    return r


class Lattice:
    """A lattice in FP64 with the 1D velocities v (D1Q5 by default; dim 2 is
    the tensor product).

    bc: 0 periodic, 1 zero-gradient ghost ends (1D only).
    theta0: None for the thermal model (the equilibrium at the local
    temperature), or the fixed reference temperature of the isothermal
    models (Sec. 2.3, Eq. 1d3v: mu_2 = theta0 + u^2)."""

    def __init__(self, dim, nx, ny=1, v=V_D1Q5, omega=1.0, bc=0, c=None, theta0=None):
        self.dim, self.nx, self.ny = int(dim), int(nx), int(ny)
        self.v = _f64(v)
        self.q1d = self.v.size
        self.q = self.q1d if self.dim == 1 else self.q1d ** 2
        self.c = lagrange_coeffs(self.v) if c is None else _f64(c)
        self.omega = float(omega)
        self.bc = int(bc)
        self.theta0 = None if theta0 is None else float(theta0)

    @property
    def shape(self):
        if self.dim == 1:
            return (self.q, self.nx)
        return (self.q, self.ny, self.nx)

    def init(self, rho, ux, uy, theta):
        """f(x, 0) = f_eq(rho, u, theta)(x)  (Eq. eqdist)."""
        f = np.zeros(self.shape)
        uy = np.zeros_like(_f64(rho)) if uy is None else uy
        if self.theta0 is not None:            # isothermal: f_eq at theta0
            theta = np.full(np.shape(rho), self.theta0)
        rc = _load().ref_init(self.dim, self.nx, self.ny, self.q1d, _p(self.v),
                              _p(self.c), _p(_f64(rho)), _p(_f64(ux)),
                              _p(_f64(uy)), _p(_f64(theta)), _p(f))
        if rc != 0:
            raise ValueError("ref_init rejected its arguments")
        return f

    def step(self, f, nsteps=1, reverse_sums=False):
        """nsteps applications of Eq. srt (push form); returns a new array."""
        g = _f64(f).copy()
        rc = _load().ref_step_theta0(self.dim, self.nx, self.ny, self.q1d, _p(self.v),
                                     _p(self.c), self.omega, self.bc,
                                     0.0 if self.theta0 is None else self.theta0, _p(g),
                                     int(nsteps), 1 if reverse_sums else 0)
        if rc != 0:
            raise ValueError("ref_step rejected its arguments")
        return g

    def moments(self, f, reverse_sums=False):
        """(rho, ux, uy, theta) of every node (discrete-moment reading)."""
        n = self.nx * self.ny
        rho, ux, uy, th = (np.zeros(n) for _ in range(4))
        f = _f64(f)
        rc = _load().ref_moments(self.dim, self.nx, self.ny, self.q1d,
                                 _p(self.v), _p(f), _p(rho), _p(ux), _p(uy),
                                 _p(th), 1 if reverse_sums else 0)
        if rc != 0:
            raise ValueError("ref_moments rejected its arguments")
        shp = (self.nx,) if self.dim == 1 else (self.ny, self.nx)
        return tuple(a.reshape(shp) for a in (rho, ux, uy, th))

    def sums(self, f):
        """Compensated (sum f, sum f vx, sum f vy, sum f |v|^2) over nodes."""
        out = np.zeros(4)
        rc = _load().ref_sums(self.dim, self.nx, self.ny, self.q1d, _p(self.v),
                              _p(_f64(f)), _p(out))
        if rc != 0:
            raise ValueError("ref_sums rejected its arguments")
        return out


class Lattice3:
    """A D3Q125 lattice (tensor product of the 1D rule over three axes,
    Sec. 2.4) in FP64, periodic.  Populations: float64 arrays of shape
    (q, nz, ny, nx), k = i + q1d j + q1d^2 l."""

    def __init__(self, nx, ny, nz, v=V_D1Q5, omega=1.0, c=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.v = _f64(v)
        self.q1d = self.v.size
        self.q = self.q1d ** 3
        self.c = lagrange_coeffs(self.v) if c is None else _f64(c)
        self.omega = float(omega)

    @property
    def shape(self):
        return (self.q, self.nz, self.ny, self.nx)

    def init(self, rho, ux, uy, uz, theta):
        """f(x, 0) = f_eq(rho, u, theta)(x)  (Eq. eqdist, three axes)."""
        f = np.zeros(self.shape)
        rc = _load().ref_init3(self.nx, self.ny, self.nz, self.q1d, _p(self.v), _p(self.c),
                               _p(_f64(rho)), _p(_f64(ux)), _p(_f64(uy)), _p(_f64(uz)),
                               _p(_f64(theta)), _p(f))
        if rc != 0:
            raise ValueError("ref_init3 rejected its arguments")
        return f

    def step(self, f, nsteps=1):
        """nsteps applications of Eq. srt (push form); returns a new array."""
        g = _f64(f).copy()
        rc = _load().ref_step3(self.nx, self.ny, self.nz, self.q1d, _p(self.v), _p(self.c),
                               self.omega, _p(g), int(nsteps))
        if rc != 0:
            raise ValueError("ref_step3 rejected its arguments")
        return g

    def moments(self, f):
        """(rho, ux, uy, uz, theta), each (nz, ny, nx); 3 rho theta = sum f |v - u|^2."""
        n = self.nx * self.ny * self.nz
        out = [np.zeros(n) for _ in range(5)]
        rc = _load().ref_moments3(self.nx, self.ny, self.nz, self.q1d, _p(self.v), _p(_f64(f)),
                                  *[_p(a) for a in out])
        if rc != 0:
            raise ValueError("ref_moments3 rejected its arguments")
        return tuple(a.reshape(self.nz, self.ny, self.nx) for a in out)

    def sums(self, f):
        """Compensated (sum f, sum f vx, sum f vy, sum f vz, sum f |v|^2)."""
        out = np.zeros(5)
        rc = _load().ref_sums3(self.nx, self.ny, self.nz, self.q1d, _p(self.v), _p(_f64(f)),
                               _p(out))
        if rc != 0:
            raise ValueError("ref_sums3 rejected its arguments")
        return out
