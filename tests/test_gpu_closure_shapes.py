"""Closure kernels at shapes whose launches exercise every path of their
blocking.  Bounds as in the closure kernel tests: FP32 accumulation of bf16
products, bf16 stores.

  * 64 x 250 nodes, 4 frames: the convolution blocks hold 3 output rows each
    (about 256 blocks: the three-row register ring runs through all of its
    phases, with its row prefetch, and the last block of a frame is ragged),
    the input-gradient blocks 1 row, and the weight-gradient blocks 16 rows
    with a ragged 10-row band at the end of each frame.  Only two of a
    convolution block's four waves have nodes (64 = 2 x 32).
  * 256 x 250 nodes, 8 frames (the width and frame count of the coarse
    256^2 training batch): two convolution blocks per row band
    (blockIdx.x > 0) with all four waves live, 15-row blocks with a ragged
    10-row band, 7-row input-gradient blocks (ragged 5), and four 64-node
    weight-gradient segments per row band.
"""
import numpy as np
import pytest
import torch

from oracle import closure as ocl
from paper_1402_5487_amd import inputs
from paper_1402_5487_amd.closure import CNN_PARAMS, Closure, init_params, split_params
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

SHAPES = [(64, 250, 4), (256, 250, 8)]
BF = 2.0 ** -8


def _conv_rows(nx, ny, frames):
    # the launch arithmetic of the convolutions (target 256 blocks, 16 rows at most)
    blocks1 = ((nx // 32 + 3) // 4) * ny * frames
    return max(1, min(16, blocks1 // 256))


def test_conv_row_blocking_matches_the_shapes():
    r0 = _conv_rows(*SHAPES[0])
    assert r0 == 3 and SHAPES[0][1] % r0 != 0 and SHAPES[0][1] % 16 != 0
    r1 = _conv_rows(*SHAPES[1])
    assert r1 == 15 and SHAPES[1][1] % r1 != 0 and SHAPES[1][1] % (r1 // 2) != 0
    assert SHAPES[1][0] // 32 // 4 == 2 and SHAPES[1][0] // 64 == 4


@pytest.fixture(scope="module", params=SHAPES, ids=lambda s: "%dx%dx%d" % s)
def run(request):
    NX, NY, FRAMES = request.param
    print(f"closure shapes {NX}x{NY}, {FRAMES} frames", flush=True)
    posts = []
    for f in range(FRAMES):
        fields = inputs.kelvin_helmholtz(NX, NY, u0=0.04 + 0.02 * f, delta=4.0, theta=0.35,
                                         mode=1 + f % 2)
        lat = Lattice(2, NX, NY, omega=1.9, storage="f64").init(*fields)
        lat.step(2 + f)
        posts.append(lat.f.clone())
    P = np.stack([p.view(NY, 25, NX).permute(0, 2, 1).double().cpu().numpy() for p in posts])
    mean = P.mean(axis=(0, 1, 2))
    scale = P.std(axis=(0, 1, 2)) + 1e-6
    g = torch.Generator(device="cuda").manual_seed(2)
    targets = [torch.randn(4, NY, NX, generator=g, device="cuda", dtype=torch.float32) * 1e-4
               for _ in range(FRAMES)]
    msig = np.full(4, 1e-4)
    oscale = 4e-4 * mean / mean.sum()
    net = Closure(NX, NY, FRAMES)
    net.set_norm(mean, scale, oscale, msig)
    params = init_params(seed=11, out_gain=1.0)
    gb = torch.Generator().manual_seed(6)
    for layer, cout in enumerate((32, 32, 25)):
        off = layer * 9248 + 9 * 32 * 32
        params[off:off + cout] = (torch.rand(cout, generator=gb) * 0.2 - 0.1).to(params.device)
    net.forward(params, posts)
    grads = torch.zeros(CNN_PARAMS, dtype=torch.float32, device="cuda")
    net.backward(params, targets, grads, reg=0.05)
    torch.cuda.synchronize()
    acts = {k: net.activation(k).double().cpu().numpy() for k in range(7)}
    return dict(params=params, pb=split_params(params.to(torch.bfloat16).float()), acts=acts,
                grads=grads.double().cpu().numpy(), frames=FRAMES)


def _conv_ok(got, x, w, b, relu, store_bf16):
    ref = ocl.conv3x3(x, w, b)
    bound = 2e-5 * ocl.conv3x3(np.abs(x), np.abs(w), np.abs(b))
    if relu:
        ref = np.maximum(ref, 0.0)
    if store_bf16:
        bound = bound + BF * np.abs(ref)
    return (np.abs(got - ref) - bound).max() <= 1e-30, float(np.abs(got - ref).max())


def test_forward_layers(run):
    a, p = run["acts"], run["params"]
    (w1, _), (w2, _), (w3, _) = run["pb"]
    b1, b2, b3 = (p[l * 9248 + 9216:l * 9248 + 9216 + c].double().cpu().numpy()
                  for l, c in ((0, 32), (1, 32), (2, 25)))
    for f in range(run["frames"]):
        for got, x, w, b, relu, bf in ((a[1][f], a[0][f][..., :25], w1, b1, True, True),
                                       (a[2][f], a[1][f], w2, b2, True, True),
                                       (a[3][f][..., :25], a[2][f], w3, b3, False, False)):
            ok, e = _conv_ok(got, x, w, b, relu, bf)
            assert ok, (f, e)


def test_backward_layers(run):
    a, g = run["acts"], run["grads"]
    (w1, _), (w2, _), (w3, _) = run["pb"]
    chain = [(a[2], w3, a[4][..., :25], a[2], 2, a[5]),
             (a[1], w2, a[5], a[1], 1, a[6]),
             (a[0][..., :25], w1, a[6], None, 0, None)]
    for x, w, dz, act_below, layer, dz_below in chain:
        dw_ref, db_ref, dw_abs = np.zeros(w.shape), np.zeros(w.shape[3]), np.zeros(w.shape)
        for f in range(run["frames"]):
            dx, dw, db = ocl.conv3x3_backward(x[f], w, dz[f])
            dabs = ocl.conv3x3_backward(np.abs(x[f]), np.abs(w), np.abs(dz[f]))
            dw_ref += dw
            db_ref += db
            dw_abs += dabs[1]
            if dz_below is not None:
                ref = dx * (act_below[f] > 0)
                bound = BF * np.abs(ref) + 2e-5 * dabs[0]
                assert (np.abs(dz_below[f] - ref) - bound).max() <= 1e-30, ("dz", layer, f)
        w_flat = g[layer * 9248:layer * 9248 + 9216].reshape(9, 32, 32)
        gw = np.transpose(w_flat, (0, 2, 1)).reshape(3, 3, 32, 32)
        gb = g[layer * 9248 + 9216:layer * 9248 + 9248]
        cin, cout = w.shape[2], w.shape[3]
        assert (np.abs(gw[:, :, :cin, :cout] - dw_ref) - 2e-4 * dw_abs).max() <= 1e-30, ("dW", layer)
        assert np.abs(gb[:cout] - db_ref).max() <= 2e-4 * np.abs(dz).sum() + 1e-12, ("db", layer)
