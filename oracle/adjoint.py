"""FP64 adjoints of the coarse step and of the closure's equilibrium shift
(TEST INFRASTRUCTURE ONLY).

Training the learned closure through several coarse steps needs the
transpose of the step's Jacobian.  This module is the plain definition the
GPU adjoint kernels are checked against; its own pins are dot-product tests
against central finite differences of the oracle's forward maps
(tests/test_oracle_adjoint.py).

Notation (node-major arrays (H, W, 25), population k = i + 5 j moving with
(v_i, v_j), the pull layout of the closure oracle):
  S = pull(P)                 pre-collision state from a post-collision buffer
  m = Phi^T S                 conserved densities (rho, j_x, j_y, E), E = sum f |v|^2
  F(m) = f_eq                 the tensor-product equilibrium of Eq. eqdist with
                              rho, u = j / rho, 2 theta = E / rho - |u|^2
  step:  P' = (1 - omega) S + omega F(m(S))          (Eq. srt, collision half)
  shift: P' = P + push(F(m + g) - F(m)),  g = pull(c) Phi - c Phi
The derivatives of F follow from r_i = sum_n c_in mu_n (Eq. rdr) and the
Maxwell moments: d mu_n / du = n mu_(n-1), d mu_n / d theta =
n (n - 1) / 2 mu_(n-2) (differentiating the Gaussian moments).
"""
import numpy as np

from . import V_D1Q5, lagrange_coeffs, maxwell_moments
from .closure import conserved_basis, pull, push


def _rule_and_derivs(c, u, theta):
    """r, dr/du, dr/dtheta of the 1D rule at (u, theta)."""
    q = c.shape[0]
    mu = maxwell_moments(u, theta, q - 1)
    du = np.array([n * mu[n - 1] if n >= 1 else 0.0 for n in range(q)])
    dt = np.array([n * (n - 1) / 2.0 * mu[n - 2] if n >= 2 else 0.0 for n in range(q)])
    return c @ mu, c @ du, c @ dt


def primitive(m):
    """(rho, u_x, u_y, theta) of conserved densities m = (rho, j_x, j_y, E)."""
    rho = m[..., 0]
    ux, uy = m[..., 1] / rho, m[..., 2] / rho
    return rho, ux, uy, 0.5 * (m[..., 3] / rho - ux * ux - uy * uy)


def equilibrium(m, c=None):
    """F(m): (..., 25) equilibrium of conserved densities m (..., 4)."""
    c = lagrange_coeffs(V_D1Q5) if c is None else c
    rho, ux, uy, th = primitive(m)
    out = np.empty(m.shape[:-1] + (25,))
    for idx in np.ndindex(m.shape[:-1]):
        rx = _rule_and_derivs(c, ux[idx], th[idx])[0]
        ry = _rule_and_derivs(c, uy[idx], th[idx])[0]
        out[idx] = rho[idx] * np.outer(ry, rx).ravel()      # [j][i] -> k = i + 5 j
    return out


def equilibrium_vjp(m, lam, c=None):
    """a = J_F(m)^T lam: (..., 4) for conserved densities m (..., 4) and
    cotangents lam (..., 25)."""
    c = lagrange_coeffs(V_D1Q5) if c is None else c
    rho, ux, uy, th = primitive(m)
    a = np.empty(m.shape[:-1] + (4,))
    for idx in np.ndindex(m.shape[:-1]):
        R, U, W, T = rho[idx], ux[idx], uy[idx], th[idx]
        rx, rxu, rxt = _rule_and_derivs(c, U, T)
        ry, ryu, ryt = _rule_and_derivs(c, W, T)
        L = lam[idx].reshape(5, 5)                            # L[j, i]
        g_rho = ry @ L @ rx                                   # sum lam r_i r_j
        g_ux = R * (ry @ L @ rxu)
        g_uy = R * (ryu @ L @ rx)
        g_th = R * (ry @ L @ rxt + ryt @ L @ rx)
        # chain rule from (rho, u_x, u_y, theta) to (rho, j_x, j_y, E)
        a[idx] = (g_rho - g_ux * U / R - g_uy * W / R + g_th * (U * U + W * W - 2 * T) / (2 * R),
                  g_ux / R - g_th * U / R,
                  g_uy / R - g_th * W / R,
                  g_th / (2 * R))
    return a


def collide(S, omega, c=None):
    """Post-collision populations of the pre-collision state S (..., 25)."""
    phi = conserved_basis()
    return (1.0 - omega) * S + omega * equilibrium(S @ phi, c)


def step(P, omega, c=None):
    """One plain step of a post-collision buffer: P' = collide(pull(P))."""
    return collide(pull(P), omega, c)


def step_vjp(P, lam, omega, c=None):
    """dL/dP for P' = step(P) and lam = dL/dP'."""
    phi = conserved_basis()
    S = pull(P)
    a = equilibrium_vjp(S @ phi, lam, c)
    return push((1.0 - omega) * lam + omega * (a @ phi.T))


def shift(P, cc, c=None):
    """The closure's apply: P' = P + push(F(m + g) - F(m)) with m the
    conserved densities of pull(P) and g = pull(cc) Phi - cc Phi (flux form)."""
    phi = conserved_basis()
    m = pull(P) @ phi
    g = pull(cc) @ phi - cc @ phi
    return P + push(equilibrium(m + g, c) - equilibrium(m, c))


def shift_vjp(P, cc, lam, c=None):
    """(dL/dP, dL/dcc) for P' = shift(P, cc) and lam = dL/dP'."""
    phi = conserved_basis()
    m = pull(P) @ phi
    g = pull(cc) @ phi - cc @ phi
    Lam = pull(lam)                                           # dL/d(shift) at each node
    a_g = equilibrium_vjp(m + g, Lam, c)
    a_m = a_g - equilibrium_vjp(m, Lam, c)
    dP = lam + push(a_m @ phi.T)
    dcc = push(a_g @ phi.T) - a_g @ phi.T
    return dP, dcc


def moment_loss(P, target_cons, weights):
    """L = (1/N) sum_x sum_j w_j (m_j(x) - target_j(x))^2 with m = Phi^T pull(P)
    (the conserved densities of the state P holds) and its gradient dL/dP."""
    phi = conserved_basis()
    r = pull(P) @ phi - target_cons
    n = P.shape[0] * P.shape[1]
    w = np.asarray(weights, dtype=np.float64)
    loss = float((w * r * r).sum() / n)
    return loss, push((2.0 / n * w * r) @ phi.T)
