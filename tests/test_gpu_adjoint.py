"""GPU adjoints for training the closure through coarse steps, against the
adjoint oracle (oracle/adjoint.py, itself pinned by dot-product tests
against finite differences of the oracle's forward maps).

Bounds: the step, loss and shift adjoints run in FP64 on both sides, in
different operation orders: 1e-12 relative to the largest value.  The
moment cotangent the network backward reads is stored in FP32 (2^-23
relative).  The network-input gradient is a bf16 MFMA convolution with FP32
accumulation: the closure kernel tests' bound 2e-5 of the sum of absolute
terms.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from oracle import closure as ocl
from paper_1402_5487_amd import _plbm, inputs
from paper_1402_5487_amd.closure import Closure, init_params, split_params
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

NX, NY, FRAMES = 64, 40, 2
OMEGA = 1.9


def _nodes(buf, ny=NY, nx=NX):
    """population-layout buffer -> float64 numpy (ny, nx, 25)"""
    return buf.view(ny, 25, nx).permute(0, 2, 1).double().cpu().numpy()


def _rows(a):
    """(ny, nx, 25) numpy -> FP64 device buffer in the population layout"""
    return torch.from_numpy(np.ascontiguousarray(np.transpose(a, (0, 2, 1)))).reshape(-1).cuda()


def _lattice(seed, storage="f64", steps=3):
    fields = inputs.random_fields(NX, NY, seed=seed, u=0.04)
    lat = Lattice(2, NX, NY, omega=OMEGA, storage=storage).init(*fields)
    lat.step(steps)
    return lat


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_step_vjp_matches_oracle(storage):
    lat = _lattice(1, storage)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal((NY, NX, 25))
    out = torch.empty(NY * 25 * NX, dtype=torch.float64, device="cuda")
    _plbm.step_vjp(lat.desc, lat.f, _rows(lam), out, lat.stream)
    want = adj.step_vjp(_nodes(lat.f), lam, OMEGA)
    assert _rel(_nodes(out), want) < 1e-12


@pytest.fixture(scope="module")
def net_setup():
    lats = [_lattice(10 + f) for f in range(FRAMES)]
    posts = [l.f.clone() for l in lats]
    P = np.stack([_nodes(p) for p in posts])
    net = Closure(NX, NY, FRAMES)
    mean = P.mean(axis=(0, 1, 2))
    scale = P.std(axis=(0, 1, 2)) + 1e-6
    msig = np.array([1e-4, 2e-4, 2e-4, 5e-4])
    oscale = 1e-3 * mean / mean.sum()
    net.set_norm(mean, scale, oscale, msig)
    params = init_params(seed=4, out_gain=1.0)
    net.forward(params, posts)
    return dict(net=net, posts=posts, P=P, mean=mean, scale=scale, msig=msig, oscale=oscale,
                params=params)


def test_rollout_loss_matches_oracle(net_setup):
    s = net_setup
    rng = np.random.default_rng(5)
    truths, cons = [], []
    for f in range(FRAMES):
        m = ocl.pull(s["P"][f]) @ ocl.conserved_basis()
        m = m + 1e-4 * rng.standard_normal(m.shape) * np.array([1, 1, 1, 3])
        prim = adj.primitive(m)
        truths.append(tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in prim))
        cons.append(m)
    lams = [torch.zeros(NY * 25 * NX, dtype=torch.float64, device="cuda") for _ in range(FRAMES)]
    scale = 1.0 / (NX * NY)
    loss = s["net"].rollout_loss(s["posts"], truths, scale, lams)
    # the loss weights as the library holds them: 1 / sigma^2 of the FP32
    # moment scales, rounded to FP32
    sig = np.float32(s["msig"]).astype(np.float64)
    w = np.float32(1.0 / sig ** 2).astype(np.float64)
    want_loss = 0.0
    for f in range(FRAMES):
        l, g = adj.moment_loss(s["P"][f], cons[f], w)
        want_loss += l
        assert _rel(_nodes(lams[f]), g) < 1e-12
    assert abs(loss / want_loss - 1) < 1e-12


def test_apply_vjp_and_network_backward_match_oracle(net_setup):
    s = net_setup
    net, params = s["net"], s["params"]
    net.forward(params, s["posts"])
    rng = np.random.default_rng(6)
    lam0 = [rng.standard_normal((NY, NX, 25)) for _ in range(FRAMES)]
    lams = [_rows(l) for l in lam0]
    net.apply_vjp(s["posts"], lams)
    C = net.activation(7).permute(0, 2, 3, 1).double().cpu().numpy()       # (f, ny, nx, 25)
    Ag = net.activation(8).permute(0, 2, 3, 1).double().cpu().numpy()      # (f, ny, nx, 4)
    phi = ocl.conserved_basis()
    for f in range(FRAMES):
        dP, _ = adj.shift_vjp(s["P"][f], C[f], lam0[f])
        assert _rel(_nodes(lams[f]), dP) < 1e-12, f
        m = ocl.pull(s["P"][f]) @ phi
        g = ocl.pull(C[f]) @ phi - C[f] @ phi
        ag = adj.equilibrium_vjp(m + g, ocl.pull(lam0[f]))
        assert np.abs(Ag[f] - ag).max() <= 2.0 ** -22 * np.abs(ag).max(), f
    # the network part: dL/dy from a_g, back through the layers, and the
    # gradient of the network input added to lam
    before = [l.clone() for l in lams]
    grads = torch.zeros(3 * 9248, dtype=torch.float32, device="cuda")
    net.backward_vjp(params, grads, accumulate=False, lams=lams)
    torch.cuda.synchronize()
    x0 = net.activation(0).double().cpu().numpy()[..., :25]
    dz1 = net.activation(6).double().cpu().numpy()
    dx = net.activation(11).double().cpu().numpy()
    (w1, _), _, _ = split_params(params.to(torch.bfloat16).float())
    w1 = w1.astype(np.float64)
    inv = 1.0 / s["scale"]
    for f in range(FRAMES):
        ref = ocl.conv3x3_backward(x0[f], w1, dz1[f])[0]
        bound = 2e-5 * ocl.conv3x3_backward(np.abs(x0[f]), np.abs(w1), np.abs(dz1[f]))[0]
        assert (np.abs(dx[f][..., :25] - ref) - bound).max() <= 1e-30, f
        added = _nodes(lams[f]) - _nodes(before[f])
        want = inv * dx[f][..., :25]
        assert np.abs(added - want).max() <= 1e-6 * np.abs(want).max() + 1e-300, f
    # the output gradient the layers start from: Ph (s * dL/dc), dL/dc the
    # push of a_g minus a_g
    dy3 = net.activation(4).double().cpu().numpy()[..., :25]
    Ph = ocl.projection(s["oscale"])
    for f in range(FRAMES):
        a = Ag[f]
        dc = ocl.push(a @ phi.T) - a @ phi.T
        dy = (s["oscale"] * dc) @ Ph
        assert np.abs(dy3[f] - dy).max() <= 2.0 ** -7 * np.abs(dy).max(), f
    assert torch.isfinite(grads).all() and float(grads.abs().max()) > 0


def test_rollout_gradient_matches_finite_differences():
    """The whole chain the closure's training uses (the loss over a segment of
    corrected steps, back through each apply, the network and the fused
    step), as a directional derivative along the last layer's weights,
    against central differences of the segment loss.  The network runs in
    bf16, so the step is large (5 % of the weights) and the bound 5 %."""
    from paper_1402_5487_amd import closure_train as ct
    n, seg, B = 64, 4, 2
    ex = ct.Experiment(n_coarse=n, factor=4, batch=B)
    ex.generate(range(2), 4, 40, rng_seed=0)
    ex.fit_norm()
    ex.fit_rollout_scale(range(2), steps=20)
    p = init_params(0, ex.device, out_gain=1.0)
    fines = [ex.fine_lattice(s) for s in (3, 4)]
    coarses = [ex.coarse_lattice().init(*ex.restricted(f)) for f in fines]
    for f, c in zip(fines, coarses):
        f.step(4 * 5)
        c.step(5)
    start = [c.f.clone() for c in coarses]
    truth = []
    for _ in range(seg):
        for f in fines:
            f.step(4)
        truth.append([ex.restricted(f) for f in fines])
    scale = 1.0 / (seg * B * n * n)

    def run(params, grad=None):
        for c, s0 in zip(coarses, start):
            c.f.copy_(s0)
        post, pre = [[c.f.clone() for c in coarses]], []
        for _ in range(seg):
            for c in coarses:
                c.step(1)
            pre.append([c.f.clone() for c in coarses])
            ex.net.forward(params, [c.f for c in coarses])
            ex.net.apply([c.f for c in coarses], bound=float("inf"))
            post.append([c.f.clone() for c in coarses])
        loss = sum(ex.net.rollout_loss(post[s], truth[s - 1], scale) for s in range(1, seg + 1))
        if grad is not None:
            lam = [torch.zeros(n * n * 25, dtype=torch.float64, device="cuda") for _ in range(B)]
            tmp = [torch.zeros_like(x) for x in lam]
            for s in range(seg, 0, -1):
                ex.net.rollout_loss(post[s], truth[s - 1], scale, lam, want_loss=False)
                ex.net.forward(params, pre[s - 1])
                ex.net.apply_vjp(pre[s - 1], lam)
                ex.net.backward_vjp(params, grad, accumulate=(s != seg), lams=lam)
                for b in range(B):
                    _plbm.step_vjp(coarses[b].desc, post[s - 1][b], lam[b], tmp[b], coarses[b].stream)
                lam, tmp = tmp, lam
        return loss

    g = torch.zeros_like(p)
    run(p, g)
    w3 = slice(2 * 9248, 2 * 9248 + 9216)
    d = torch.zeros_like(p)
    d[w3] = torch.randn(9216, generator=torch.Generator(device="cuda").manual_seed(9),
                        device="cuda") * p[w3].abs().max()
    h = 0.05
    fd = (run(p + h * d) - run(p - h * d)) / (2 * h)
    adj_dir = float((g * d).sum())
    assert abs(fd / adj_dir - 1) < 0.05, (fd, adj_dir)
