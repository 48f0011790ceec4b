"""FP64 reference of the learned closure (TEST INFRASTRUCTURE ONLY).

The closure is the learned form of the build: a 3-layer 3x3 convolutional
network that maps a coarse lattice's normalised post-collision populations to
a correction of them.  The paper has no such network; this module is the
plain, slow definition the GPU kernels are checked against:

  conv3x3 with periodic padding:
      out[y, x, o] = b[o] + sum_{dy, dx in {-1, 0, 1}} sum_i
                     in[(y + dy) mod H, (x + dx) mod W, i] * w[dy + 1, dx + 1, i, o]
  network: conv(25 -> 32), ReLU, conv(32 -> 32), ReLU, conv(32 -> 25)
  projection (normalised coordinates, output scales s): with
      B = diag(s) Phi, Phi_k = (1, v_x, v_y, |v|^2) of the D2Q25 velocities,
      Ph = I - B (B^T B)^-1 B^T, so the physical correction c = s * (Ph y)
      has zero mass, momentum and energy at every node (the invariants of
      Eq. srt); it is the closest such vector in the metric sum_k (x_k / s_k)^2
  loss (moment form): the corrected buffer P + c is streamed (pull form,
      f_k(x) = P_k(x - v_k)) and its conserved densities (rho, j_x, j_y, E)
      are compared with a target (flux form: Phi^T (pull(c) - c), the same for
      a moment-free c); since streaming and the moments are linear
      and P's own contribution is known, the target is handed over as the
      increment error d = (truth increment) - (plain-step increment) and
      L = mean over nodes of sum_m ((Phi^T pull(c))_m - d_m)^2 / sigma_m^2
          + beta |Ph y|^2 (minimum-norm term)
  apply: the streamed moments g of the correction are handed to the next
      step as a shift f_eq(m + g) - f_eq(m) of its pulled populations, which
      keeps their non-equilibrium part
  Adam (Kingma & Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
      p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
  restriction: 4 x 4 block means of rho, rho u and sum f |v|^2.

Arrays are float64 numpy, images (H, W, C).
"""
import numpy as np

V5 = np.array([0.0, 1.0, -1.0, 3.0, -3.0])


def velocities_2d():
    """(25, 2) velocities of population k = i + 5 j."""
    return np.array([[V5[k % 5], V5[k // 5]] for k in range(25)])


def conserved_basis():
    """Phi (25 x 4): 1, v_x, v_y, |v|^2 at each velocity."""
    v = velocities_2d()
    return np.stack([np.ones(25), v[:, 0], v[:, 1], (v ** 2).sum(1)], axis=1)


def projection(scale=None):
    """Ph (25 x 25) in normalised coordinates for output scales `scale`
    (all ones: the Euclidean projection)."""
    s = np.ones(25) if scale is None else np.asarray(scale, dtype=np.float64)
    B = s[:, None] * conserved_basis()
    return np.eye(25) - B @ np.linalg.solve(B.T @ B, B.T)


def conv3x3(x, w, b):
    """Periodic 3x3 convolution (cross-correlation), written out."""
    H, W, _ = x.shape
    out = np.broadcast_to(b, (H, W, w.shape[3])).astype(np.float64).copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            shifted = np.roll(x, shift=(-dy, -dx), axis=(0, 1))   # shifted[y,x] = x[y+dy, x+dx]
            out += shifted @ w[dy + 1, dx + 1]
    return out


def conv3x3_backward(x, w, dout):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for dy in (-1, 0, 1):
        for ddx in (-1, 0, 1):
            shifted = np.roll(x, shift=(-dy, -ddx), axis=(0, 1))
            dw[dy + 1, ddx + 1] = np.einsum("yxi,yxo->io", shifted, dout)
            # out[y,x] gets x[y+dy, x+dx] w  =>  dx[y', x'] += dout[y'-dy, x'-dx] w^T
            dx += np.roll(dout @ w[dy + 1, ddx + 1].T, shift=(dy, ddx), axis=(0, 1))
    return dx, dw, dout.sum(axis=(0, 1))


def forward(params, x):
    """params: list of three (w, b); returns (y, cache)."""
    (w1, b1), (w2, b2), (w3, b3) = params
    z1 = conv3x3(x, w1, b1)
    a1 = np.maximum(z1, 0.0)
    z2 = conv3x3(a1, w2, b2)
    a2 = np.maximum(z2, 0.0)
    y = conv3x3(a2, w3, b3)
    return y, (x, z1, a1, z2, a2)


def backward(params, cache, dy):
    (w1, _), (w2, _), (w3, _) = params
    x, z1, a1, z2, a2 = cache
    da2, dw3, db3 = conv3x3_backward(a2, w3, dy)
    dz2 = da2 * (z2 > 0)
    da1, dw2, db2 = conv3x3_backward(a1, w2, dz2)
    dz1 = da1 * (z1 > 0)
    _, dw1, db1 = conv3x3_backward(x, w1, dz1)
    return [(dw1, db1), (dw2, db2), (dw3, db3)]


def pull(P):
    """Streaming in the pull form with periodic wrap: f_k(y, x) =
    P_k(y - v_y, x - v_x) (Eq. srt's x + v_i dt target, read backwards)."""
    v = velocities_2d().astype(int)
    out = np.empty_like(P)
    for k in range(25):
        out[..., k] = np.roll(P[..., k], shift=(v[k, 1], v[k, 0]), axis=(0, 1))
    return out


def push(h):
    """Adjoint of pull: g_k(y, x) = h_k(y + v_y, x + v_x)."""
    v = velocities_2d().astype(int)
    out = np.empty_like(h)
    for k in range(25):
        out[..., k] = np.roll(h[..., k], shift=(-v[k, 1], -v[k, 0]), axis=(0, 1))
    return out


def streamed_moments(c):
    """Conserved densities a correction c brings to each node after
    streaming, in flux form: Phi^T (pull(c)(x) - c(x)).  For c without mass,
    momentum and energy at every node the second term is zero; written this
    way the domain totals of the result vanish for any c."""
    phi = conserved_basis()
    return pull(c) @ phi - c @ phi


def conserved(rho, ux, uy, theta):
    """(rho, rho u_x, rho u_y, E) with E = sum_k f_k |v_k|^2 = rho (2 theta +
    |u|^2) in two dimensions (d rho theta = sum f |v - u|^2, Sec. 2)."""
    return np.stack([rho, rho * ux, rho * uy, rho * (2.0 * theta + ux * ux + uy * uy)], axis=-1)


def increment_error(truth_prev, truth_now, model_prev, model_now):
    """Target of the moment loss: the one-step change of the conserved
    densities of the truth minus that of the plain coarse step; each
    argument is a (rho, ux, uy, theta) tuple of (H, W) arrays."""
    return ((conserved(*truth_now) - conserved(*truth_prev)) -
            (conserved(*model_now) - conserved(*model_prev)))


def moment_loss_and_grad(y, d, scale, mscale, reg=0.0):
    """Moment-form loss and its gradient w.r.t. the network output y.
    y: (H, W, 25); d: (H, W, 4) increment error; scale: (25,) s_k;
    mscale: (4,) sigma_m; reg: weight beta of the minimum-norm term
    beta * mean |Ph y|^2 (the moments fix 4 of the 21 free components of a
    node's correction; the term picks the smallest one that explains them).
    Returns (loss, dy, c, a) with c the physical correction and a = dL/dm
    the per-node moment residual weights."""
    s = np.asarray(scale, dtype=np.float64)
    w2 = 1.0 / np.asarray(mscale, dtype=np.float64) ** 2
    P = projection(s)
    phi = conserved_basis()
    py = y @ P.T
    c = s * py
    r = streamed_moments(c) - d
    n = y.shape[0] * y.shape[1]
    loss = ((w2 * r * r).sum() + reg * (py * py).sum()) / n
    a = 2.0 * w2 * r / n
    g = push(a @ phi.T) - a @ phi.T
    dy = (s * g) @ P + 2.0 * reg / n * py
    return loss, dy, c, a


def equilibrium_shift(P, c, lattice):
    """Apply: the correction's streamed moments g = pull(c) Phi enter the
    next step as a shift of the equilibrium (Eq. eqdist) of the pulled
    populations f = pull(P):  f + f_eq(m + g) - f_eq(m),  m the node moments
    of f; returned in the pull layout (P + push(shift)).  A node whose
    shifted density or temperature is not positive is left unshifted.
    lattice: an oracle Lattice of the same shape (D2Q25)."""
    nodes = lambda a: np.ascontiguousarray(np.transpose(a, (2, 0, 1)))
    back = lambda a: np.transpose(a, (1, 2, 0))
    rho, ux, uy, th = lattice.moments(nodes(pull(P)))
    cons = conserved(rho, ux, uy, th) + streamed_moments(c)
    r1 = cons[..., 0]
    u1, w1 = cons[..., 1] / r1, cons[..., 2] / r1
    t1 = 0.5 * (cons[..., 3] / r1 - u1 * u1 - w1 * w1)
    ok = (r1 > 0) & (t1 > 0)
    r1, u1, w1, t1 = (np.where(ok, a, b) for a, b in ((r1, rho), (u1, ux), (w1, uy), (t1, th)))
    shift = back(lattice.init(r1, u1, w1, t1)) - back(lattice.init(rho, ux, uy, th))
    return P + push(shift)


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def restrict(rho, jx, jy, e, factor=4):
    """Block means of the conserved fields; returns coarse (rho, ux, uy,
    theta) with 2 rho theta = E - rho |u|^2 (two dimensions)."""
    def bm(a):
        H, W = a.shape
        return a.reshape(H // factor, factor, W // factor, factor).mean(axis=(1, 3))
    r, X, Y, E = bm(rho), bm(jx), bm(jy), bm(e)
    ux, uy = X / r, Y / r
    return r, ux, uy, (E / r - ux * ux - uy * uy) / 2.0
