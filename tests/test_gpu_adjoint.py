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


class _Segment:
    """A segment of corrected coarse steps beside restricted fine runs (n^2
    coarse, B runs on fine seeds 3 .. 3 + B - 1), its loss and its gradient
    through every step, by the building-block calls or by the fused
    plbm_closure_rollout_vjp."""

    def __init__(self, n=64, seg=4, B=2, storage="f64"):
        from paper_1402_5487_amd import closure_train as ct
        self.n, self.seg, self.B = n, seg, B
        ex = ct.Experiment(n_coarse=n, factor=4, batch=B, storage=storage)
        ex.generate(range(2), 4, 40, rng_seed=0)
        ex.fit_norm()
        ex.fit_rollout_scale(range(2), steps=20)
        self.ex = ex
        fines = [ex.fine_lattice(s) for s in range(3, 3 + B)]
        self.coarses = [ex.coarse_lattice().init(*ex.restricted(f)) for f in fines]
        for f, c in zip(fines, self.coarses):
            f.step(4 * 5)
            c.step(5)
        self.start = [c.f.clone() for c in self.coarses]
        self.truth = []
        for _ in range(seg):
            for f in fines:
                f.step(4)
            self.truth.append([ex.restricted(f) for f in fines])
        self.scale = 1.0 / (seg * B * n * n)

    def forward(self, params):
        ex, cs = self.ex, self.coarses
        for c, s0 in zip(cs, self.start):
            c.f.copy_(s0)
        self.post, self.pre = [[c.f.clone() for c in cs]], []
        for _ in range(self.seg):
            for c in cs:
                c.step(1)
            self.pre.append([c.f.clone() for c in cs])
            ex.net.forward(params, [c.f for c in cs])
            ex.net.apply([c.f for c in cs], bound=float("inf"))
            self.post.append([c.f.clone() for c in cs])

    def loss(self, params):
        self.forward(params)
        return sum(self.ex.net.rollout_loss(self.post[s], self.truth[s - 1], self.scale)
                   for s in range(1, self.seg + 1))

    def grad(self, params, fused, keep=None):
        """Gradient into a new tensor (after forward(params)); keep, if a
        list, receives dL/dQ_(s-1) for s = seg .. 2.  Returns (grad, loss)."""
        ex, cs, B, n = self.ex, self.coarses, self.B, self.n
        g = torch.zeros(3 * 9248, dtype=torch.float32, device="cuda")
        lam = [torch.zeros(n * n * 25, dtype=torch.float64, device="cuda") for _ in range(B)]
        tmp = [torch.zeros_like(x) for x in lam]
        loss = 0.0
        for s in range(self.seg, 0, -1):
            if fused:
                ex.net.forward(params, self.pre[s - 1])
                got = ex.net.rollout_vjp(
                    cs[0].desc, params, g, s != self.seg, self.post[s], self.truth[s - 1], self.scale,
                    self.pre[s - 1], before=self.post[s - 1] if s > 1 else None,
                    lam_in=lam if s != self.seg else None, lam_out=tmp if s > 1 else None,
                    want_loss=(s == 1))
                if s == 1:
                    loss = got
            else:
                loss += ex.net.rollout_loss(self.post[s], self.truth[s - 1], self.scale, lam)
                ex.net.forward(params, self.pre[s - 1])
                ex.net.apply_vjp(self.pre[s - 1], lam)
                ex.net.backward_vjp(params, g, accumulate=(s != self.seg), lams=lam)
                if s > 1:
                    for b in range(B):
                        _plbm.step_vjp(cs[b].desc, self.post[s - 1][b], lam[b], tmp[b], cs[b].stream)
            if s > 1:
                if keep is not None:
                    keep.append([t.clone() for t in tmp])
                lam, tmp = tmp, lam
        return g, loss


@pytest.mark.parametrize("storage,n,B", [("f64", 64, 2), ("f32", 64, 2),
                                         ("f32", 256, 8)])   # the shipped training's frames
def test_fused_rollout_step_matches_the_building_blocks(storage, n, B):
    """plbm_closure_rollout_vjp against the sequence rollout_loss, apply_vjp,
    backward_vjp, step_vjp it fuses: the same terms (the loss's and the
    apply's moment cotangents summed per node before the push rather than
    pushed one after the other), so the FP64 adjoints of every step agree
    to the last bits (1e-15 of the largest value), the FP32 parameter
    gradient to 1e-6 (a last-bit change of
    an FP64 cotangent can move an FP32 rounding), and the segment loss,
    summed block by block over the steps rather than step by step, to
    1e-13.  The last case is the shape the shipped training runs: 256^2
    frames, eight of them in each launch (grid z up to 7)."""
    sg = _Segment(n=n, seg=3, B=B, storage=storage)
    p = init_params(0, "cuda", out_gain=1.0)
    sg.forward(p)
    keep_a, keep_b = [], []
    ga, la = sg.grad(p, fused=False, keep=keep_a)
    gb, lb = sg.grad(p, fused=True, keep=keep_b)
    assert len(keep_a) == len(keep_b) == 2
    for ka, kb in zip(keep_a, keep_b):
        for a, b in zip(ka, kb):
            assert float((a - b).abs().max()) <= 1e-15 * float(a.abs().max()), storage
    assert float((ga - gb).abs().max()) <= 1e-6 * float(ga.abs().max()), storage
    assert abs(lb / la - 1) < 1e-13, (la, lb)


@pytest.mark.parametrize("fused", [False, True])
def test_rollout_gradient_matches_finite_differences(fused):
    """The whole chain the closure's training uses (the loss over a segment of
    corrected steps, back through each apply, the network and the fused
    step), as a directional derivative along the last layer's weights,
    against central differences of the segment loss; by the building-block
    calls and by the fused backward step.  The network runs in bf16, so the
    step is large (5 % of the weights) and the bound 5 %."""
    sg = _Segment()
    p = init_params(0, "cuda", out_gain=1.0)
    sg.forward(p)
    g, _ = sg.grad(p, fused)
    w3 = slice(2 * 9248, 2 * 9248 + 9216)
    d = torch.zeros_like(p)
    d[w3] = torch.randn(9216, generator=torch.Generator(device="cuda").manual_seed(9),
                        device="cuda") * p[w3].abs().max()
    h = 0.05
    fd = (sg.loss(p + h * d) - sg.loss(p - h * d)) / (2 * h)
    adj_dir = float((g * d).sum())
    assert abs(fd / adj_dir - 1) < 0.05, (fd, adj_dir)


def test_fused_rollout_step_rejects_a_mismatched_lattice():
    """The descriptor must be the closure's coarse lattice (shape, storage)."""
    sg = _Segment(seg=1)
    p = init_params(0, "cuda", out_gain=1.0)
    sg.forward(p)
    g = torch.zeros(3 * 9248, dtype=torch.float32, device="cuda")
    other = _plbm.desc_default(2, 32, 64, 1.9, "f64")
    with pytest.raises(_plbm.PlbmError):
        sg.ex.net.rollout_vjp(other, p, g, False, sg.post[1], sg.truth[0], sg.scale, sg.pre[0])
    wrong_storage = _plbm.desc_default(2, 64, 64, 1.9, "f32")
    with pytest.raises(_plbm.PlbmError):
        sg.ex.net.rollout_vjp(wrong_storage, p, g, False, sg.post[1], sg.truth[0], sg.scale, sg.pre[0])
