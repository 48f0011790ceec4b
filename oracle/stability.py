"""Von Neumann (linear) stability of the SRT update around a uniform state.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Linearising Eq. srt around a
uniform equilibrium f0 gives, for a Fourier mode exp(i kappa . x), the
amplification matrix G(kappa) = diag(exp(-i kappa . v_k)) J with
J = (1 - omega) I + omega d f_eq / d f.  The Jacobian is taken by central
differences through the oracle's own moments and equilibrium, so no second
copy of the equilibrium formula exists here.  The largest |eigenvalue| over a
kappa grid tells whether round-off grows (> 1) or decays.

For its thermal KH run the paper remarks only that omega = 1.9 lies near the
largest stable value (Sec. 4); the analysis makes that quantitative for any
(theta, u, omega).
"""
import numpy as np

from . import Lattice


def _feq_of_f(lat, f):
    """One-node collision input -> its equilibrium, via the oracle."""
    one = Lattice(lat.dim, 1, 1, lat.v, lat.omega, 0, lat.c)
    shaped = f.reshape(one.shape)
    rho, ux, uy, th = one.moments(shaped)
    return one.init(rho.ravel(), ux.ravel(), uy.ravel(), th.ravel()).ravel()


def jacobian(lat, rho, ux, uy, theta, h=1e-6):
    one = Lattice(lat.dim, 1, 1, lat.v, lat.omega, 0, lat.c)
    f0 = one.init(np.array([rho]), np.array([ux]), np.array([uy]),
                  np.array([theta])).ravel()
    q = f0.size
    d = np.zeros((q, q))
    for m in range(q):
        e = np.zeros(q)
        e[m] = h
        d[:, m] = (_feq_of_f(lat, f0 + e) - _feq_of_f(lat, f0 - e)) / (2 * h)
    return (1.0 - lat.omega) * np.eye(q) + lat.omega * d


def max_amplification(lat, rho, ux, uy, theta, nk=32):
    """max |lambda| of G(kappa) over an nk x nk (2D) or nk (1D) grid of
    wave vectors in [-pi, pi)."""
    J = jacobian(lat, rho, ux, uy, theta)
    q1d = lat.q1d
    vx = np.array([lat.v[k % q1d] for k in range(lat.q)])
    vy = np.array([lat.v[k // q1d] for k in range(lat.q)]) if lat.dim == 2 \
        else np.zeros(lat.q)
    ks = -np.pi + 2 * np.pi * np.arange(nk) / nk
    kys = ks if lat.dim == 2 else np.zeros(1)
    kx, ky = np.meshgrid(ks, kys, indexing="ij")
    phase = np.exp(-1j * (kx.reshape(-1, 1) * vx + ky.reshape(-1, 1) * vy))
    # all wave vectors at once: G(kappa) = diag(phase(kappa)) J
    return float(np.abs(np.linalg.eigvals(phase[:, :, None] * J[None])).max())
