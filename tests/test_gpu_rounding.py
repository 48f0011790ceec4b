"""Stochastic rounding of the 16-bit deviations, checked one store at a time.

A uniform lattice off equilibrium gives every node the same FP32
post-collision population, so the node-to-node spread of what a step stores
comes from the rounding alone.  The FP32 value v of each plane's deviation
comes from an FP32-storage lattice stepped from the same decoded state (the
16-bit forms and the FP32 form share the FP32 collision, so this is the
value the 16-bit kernel rounds; round to nearest must agree with it).

Stochastic rounding (the hardware conversion fed with the hash of node,
population and value) must store one of v's two neighbours lo < v < hi at
every node, hi with probability (v - lo) / (hi - lo): over M nodes the mean
stored deviation is v within the standard error of a two-point draw,
(hi - lo) sqrt(p (1 - p) / M).  Round to nearest, the control, stores the
nearer neighbour everywhere, a bias far outside that bound on most planes.
"""
import numpy as np
import pytest
import torch

from helpers import decode, rest_weights
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

N = 512                      # 262,144 nodes per plane


def _planes(lat):
    """stored deviations, float64 (N, 25, N) on the host"""
    return lat.f.view(N, 25, N).double().cpu().numpy()


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_stochastic_rounding_is_unbiased_store_by_store(storage):
    th = 0.35
    ones = np.ones((N, N))
    fields = (ones, 0.02 * ones, -0.01 * ones, 0.36 * ones)
    # the initial state comes from the round-to-nearest lattice: with
    # stochastic rounding the initialisation's own stores differ node by node
    nr = Lattice(2, N, N, omega=1.3, storage=storage, theta0=th).init(*fields)
    sr = Lattice(2, N, N, omega=1.3, storage=storage, theta0=th, rounding="stochastic").init(*fields)
    assert [sr.desc.scale[k] for k in range(25)] == [nr.desc.scale[k] for k in range(25)]
    # off equilibrium: every plane's deviation moved by its own constant
    shift = torch.tensor(np.random.default_rng(11).uniform(-40.0, 40.0, 25), dtype=torch.float32,
                         device=nr.f.device)
    h = nr.f.view(N, 25, N)
    h.copy_((h.float() + shift[None, :, None]).to(h.dtype))
    assert torch.equal(h, h[:1, :, :1].expand(N, 25, N))
    sr.f.copy_(nr.f)
    ref = Lattice(2, N, N, omega=1.3, storage="f32")
    ref.f.copy_(torch.from_numpy(decode(sr.f, sr).astype(np.float32)))
    for lat in (sr, nr, ref):
        lat.step(1)

    fstar = ref.f.view(N, 25, N)
    assert torch.equal(fstar, fstar[:1, :, :1].expand(N, 25, N)), "the FP32 step is not uniform"
    w = rest_weights(th)
    base = np.array([w[k % 5] * w[k // 5] for k in range(25)], dtype=np.float32).astype(np.float64)
    scale = np.array([sr.desc.scale[k] for k in range(25)], dtype=np.float64)
    v = (fstar[0, :, 0].double().cpu().numpy() - base) / scale

    got, near = _planes(sr), _planes(nr)
    M = N * N
    far = 0
    for k in range(25):
        vals = np.unique(got[:, k, :])
        nk = np.unique(near[:, k, :])
        assert len(nk) == 1, (k, nk)
        if len(vals) == 1:                     # v itself is representable
            assert abs(vals[0] - v[k]) <= 2.0 ** -20 * abs(v[k]) and nk[0] == vals[0], (k, vals, v[k])
            continue
        assert len(vals) == 2, (k, vals)
        lo, hi = vals
        ulp = hi - lo
        assert lo < v[k] < hi, (k, lo, v[k], hi)
        # both neighbours are adjacent in the format: round to nearest picks one of them
        assert nk[0] in (lo, hi) and abs(nk[0] - v[k]) <= 0.5 * ulp * (1 + 1e-6), (k, nk, v[k])
        p = (v[k] - lo) / ulp
        phat = float((got[:, k, :] == hi).mean())
        sigma = np.sqrt(max(p * (1 - p), 1.0 / M) / M)
        assert abs(phat - p) <= 6 * sigma + 2.0 ** -12, (k, phat, p, sigma)
        if abs(nk[0] - v[k]) / ulp > 6 * sigma + 2.0 ** -12:
            far += 1
    # the control: round to nearest is biased well beyond the bound on most planes
    assert far >= 15, far
