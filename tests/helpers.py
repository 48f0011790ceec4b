"""Shared test helpers: layout conversions between the GPU library's pull-scheme
buffers and the oracle's pre-collision arrays (index bookkeeping only)."""
import numpy as np

V5 = (0, 1, -1, 3, -3)


def rest_weights(theta0):
    """r_i(u = 0, theta0) for {0, +-1, +-3}, from the oracle."""
    import oracle
    return oracle.weights_1d(oracle.lagrange_coeffs(oracle.V_D1Q5), 0.0, theta0)


def decode(buf, lat):
    """Raw device buffer -> float64 numpy array of stored populations."""
    import torch
    h = buf.detach().to("cpu")
    if h.dtype in (torch.float64, torch.float32):
        return h.double().numpy()
    d = lat.desc
    w = rest_weights(d.theta0)
    base = np.array([d.rho0 * w[k % 5] * w[k // 5] for k in range(25)],
                    dtype=np.float32).astype(np.float64)
    scale = np.array([d.scale[k] for k in range(25)], dtype=np.float64)
    g = h.float().double().numpy().reshape(lat.ny, 25, lat.nx)
    return (base[None, :, None] + scale[None, :, None] * g).ravel()


def pulled_state(buf, lat):
    """Pre-collision state f_k(x) = buffer_k(x - v_k), shaped like the oracle
    arrays ((25, ny, nx) or (5, nx))."""
    a = decode(buf, lat)
    if lat.dim == 2:
        # device layout: (y * 25 + k) * nx + x
        a = a.reshape(lat.ny, 25, lat.nx).transpose(1, 0, 2)
        out = np.empty_like(a)
        for k in range(25):
            out[k] = np.roll(a[k], (V5[k // 5], V5[k % 5]), axis=(0, 1))
        return out
    a = a.reshape(5, lat.nx + 6)
    x = np.arange(lat.nx)
    return np.stack([a[k, x + 3 - V5[k]] for k in range(5)])


def pulled_state3(buf, lat):
    """D3Q125: pre-collision state (125, nz, ny, nx) of a device buffer laid
    out as ((z * ny + y) * 125 + k) * nx + x, k = i + 5 j + 25 l."""
    a = buf.detach().to("cpu").double().numpy()
    a = a.reshape(lat.nz, lat.ny, 125, lat.nx).transpose(2, 0, 1, 3)
    out = np.empty_like(a)
    for k in range(125):
        i, j, l = k % 5, (k // 5) % 5, k // 25
        out[k] = np.roll(a[k], (V5[l], V5[j], V5[i]), axis=(0, 1, 2))
    return out


def rel_err(a, b, floor=1.0):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))
