"""GPU tests of the learned closure kernels against the FP64 closure oracle.

Each layer is checked in isolation on the GPU's own (bf16) inputs, so the
only differences are the kernel's arithmetic:
  * products of bf16 values are exact in FP32; a sum of K of them accumulated
    in FP32 is off by at most ~K * 2^-24 * sum|terms| (bound used: 2e-5 *
    sum|terms| for the K = 288 convolutions, 2e-4 for the weight gradients
    that sum 1024 nodes per block);
  * results stored as bf16 (hidden activations, gradients) add half an ulp,
    2^-9 relative (bound used: 2^-8 |value|).
"""
import numpy as np
import pytest
import torch

from oracle import closure as ocl
from paper_1402_5487_amd import inputs
from paper_1402_5487_amd.closure import (CNN_PARAMS, Closure, init_params, restrict, split_params,
                                         target)
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

N, FRAMES = 64, 2
REG = 0.05
GAIN_MIN = 0.25    # measured 0.455 on these seeds
BF = 2.0 ** -8


def _nodes(buf, n=N):
    """population buffer (row layout) -> float64 (ny, nx, 25)"""
    return buf.view(n, 25, n).permute(0, 2, 1).double().cpu().numpy()


def _bf16(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.bfloat16).double().numpy()


def _fields(rng, n, amp):
    return tuple(torch.from_numpy(a).cuda() for a in (
        1 + amp * rng.standard_normal((n, n)), amp * rng.standard_normal((n, n)),
        amp * rng.standard_normal((n, n)), 0.35 + amp * rng.standard_normal((n, n))))


@pytest.fixture(scope="module")
def setup():
    posts, targets = [], []
    rng = np.random.default_rng(8)
    for f in range(FRAMES):
        fields = inputs.kelvin_helmholtz(N, N, u0=0.05 + 0.03 * f, delta=3.0, theta=0.35)
        lat = Lattice(2, N, N, omega=1.9, storage="f64").init(*fields)
        lat.step(3)
        posts.append(lat.f.clone())
        targets.append(target(*[_fields(rng, N, 1e-3) for _ in range(4)]))
    P = np.stack([_nodes(p) for p in posts])
    D = np.stack([t.permute(1, 2, 0).double().cpu().numpy() for t in targets])
    mean = P.mean(axis=(0, 1, 2))
    scale = P.std(axis=(0, 1, 2)) + 1e-6
    msig = np.sqrt((D ** 2).mean(axis=(0, 1, 2)))
    oscale = 4 * np.sqrt((msig ** 2).mean()) * mean / mean.sum()
    net = Closure(N, N, FRAMES)
    net.set_norm(mean, scale, oscale, msig)
    params = init_params(seed=3, out_gain=1.0)
    # non-zero biases on the real channels
    g = torch.Generator().manual_seed(5)
    for layer, cout in enumerate((32, 32, 25)):
        off = layer * 9248 + 9 * 32 * 32
        params[off:off + cout] = (torch.rand(cout, generator=g) * 0.2 - 0.1).to(params.device)
    net.forward(params, posts)
    grads = torch.zeros(CNN_PARAMS, dtype=torch.float32, device="cuda")
    loss = net.backward(params, targets, grads, reg=REG)
    torch.cuda.synchronize()
    pb = split_params(params.to(torch.bfloat16).float())       # the kernels' bf16 weights
    acts = {k: net.activation(k).double().cpu().numpy() for k in range(9)}
    return dict(net=net, posts=posts, targets=targets, P=P, D=D, mean=mean, scale=scale,
                oscale=oscale, msig=msig, params=params, pb=pb, acts=acts, loss=loss,
                grads=grads.double().cpu().numpy())


def _conv_ok(got, x, w, b, relu, store_bf16):
    ref = ocl.conv3x3(x, w, b)
    bound = 2e-5 * ocl.conv3x3(np.abs(x), np.abs(w), np.abs(b))
    if relu:
        ref = np.maximum(ref, 0.0)
    if store_bf16:
        bound = bound + BF * np.abs(ref)
    err = np.abs(got - ref) - bound
    return err.max() <= 1e-30, float(np.abs(got - ref).max())


def test_input_normalisation(setup):
    x0 = setup["acts"][0]
    X = (setup["P"] - setup["mean"]) / setup["scale"]
    assert np.abs(x0[..., :25] - X).max() <= BF * np.abs(X).max() + 1e-6
    assert np.all(x0[..., 25:] == 0)


def test_input_noise_is_added_to_the_normalised_input(setup):
    net = setup["net"]
    g = torch.Generator(device="cuda").manual_seed(9)
    noise = torch.randn(FRAMES * N * N * 25, generator=g, device="cuda", dtype=torch.float32)
    net.forward(setup["params"], setup["posts"], noise, 0.25)
    x0 = net.activation(0).double().cpu().numpy()
    # noise planes [frame][k][y][x]
    nz = noise.double().cpu().numpy().reshape(FRAMES, 25, N, N).transpose(0, 2, 3, 1)
    X = (setup["P"] - setup["mean"]) / setup["scale"] + 0.25 * nz
    assert np.abs(x0[..., :25] - X).max() <= BF * np.abs(X).max() + 1e-6
    assert np.all(x0[..., 25:] == 0)
    net.forward(setup["params"], setup["posts"])            # leave the clean activations


def test_forward_layers(setup):
    a = setup["acts"]
    (w1, b1), (w2, b2), (w3, b3) = setup["pb"]
    b1, b2, b3 = (setup["params"][l * 9248 + 9216:l * 9248 + 9216 + c].double().cpu().numpy()
                  for l, c in ((0, 32), (1, 32), (2, 25)))
    for f in range(FRAMES):
        ok, e = _conv_ok(a[1][f], a[0][f][..., :25], w1, b1, True, True)
        assert ok, ("layer1", e)
        ok, e = _conv_ok(a[2][f], a[1][f], w2, b2, True, True)
        assert ok, ("layer2", e)
        ok, e = _conv_ok(a[3][f][..., :25], a[2][f], w3, b3, False, False)
        assert ok, ("layer3", e)


def test_loss_and_output_gradient(setup):
    """The kernels' loss averages over all frames' nodes: the oracle's
    per-frame loss and gradients are divided by the frame count."""
    a = setup["acts"]
    loss = 0.0
    for f in range(FRAMES):
        y = a[3][f][..., :25]
        lf, dy, c, am = ocl.moment_loss_and_grad(y, setup["D"][f], setup["oscale"], setup["msig"], REG)
        loss += lf / FRAMES
        got_c = np.transpose(a[7][f], (1, 2, 0))
        assert np.abs(got_c - c).max() <= 1e-5 * np.abs(c).max()
        got_a = np.transpose(a[8][f], (1, 2, 0))
        ref_a = am / FRAMES
        assert np.abs(got_a - ref_a).max() <= 1e-4 * np.abs(ref_a).max()
        ref = dy / FRAMES
        got = a[4][f][..., :25]
        assert (np.abs(got - ref) - BF * np.abs(ref) - 1e-4 * np.abs(ref).max()).max() <= 0
    assert abs(setup["loss"] / loss - 1) < 1e-4
    assert np.all(a[4][..., 25:] == 0)


def test_target_matches_oracle():
    rng = np.random.default_rng(21)
    groups = [_fields(rng, 40, 0.05) for _ in range(4)]
    got = target(*groups).permute(1, 2, 0).double().cpu().numpy()
    ref = ocl.increment_error(*[tuple(t.cpu().numpy() for t in g) for g in groups])
    # FP64 arithmetic rounded once to FP32
    assert np.abs(got - ref).max() <= 2.0 ** -24 * np.abs(ref).max() * 2


def _grad_layer(g, layer, cin, cout):
    w = g[layer * 9248:layer * 9248 + 9216].reshape(9, 32, 32)      # [t][o][i]
    b = g[layer * 9248 + 9216:layer * 9248 + 9248]
    return np.transpose(w, (0, 2, 1)).reshape(3, 3, 32, 32), b


def test_backward_layers(setup):
    a, pb, g = setup["acts"], setup["pb"], setup["grads"]
    (w1, _), (w2, _), (w3, _) = pb
    # (input activation, weights, upstream gradient, next-lower activation, layer)
    chain = [(a[2], w3, a[4][..., :25], a[2], 2, a[5]),
             (a[1], w2, a[5], a[1], 1, a[6]),
             (a[0][..., :25], w1, a[6], None, 0, None)]
    for x, w, dz, act_below, layer, dz_below in chain:
        dw_ref = np.zeros(w.shape)
        db_ref = np.zeros(w.shape[3])
        dw_abs = np.zeros(w.shape)
        for f in range(FRAMES):
            dx, dw, db = ocl.conv3x3_backward(x[f], w, dz[f])
            dw_ref += dw
            db_ref += db
            dw_abs += ocl.conv3x3_backward(np.abs(x[f]), np.abs(w), np.abs(dz[f]))[1]
            if dz_below is not None:
                ref = dx * (act_below[f] > 0)
                bound = BF * np.abs(ref) + 2e-5 * ocl.conv3x3_backward(
                    np.abs(x[f]), np.abs(w), np.abs(dz[f]))[0]
                assert (np.abs(dz_below[f] - ref) - bound).max() <= 1e-30, ("dz", layer)
        gw, gb = _grad_layer(g, layer, w.shape[2], w.shape[3])
        cin, cout = w.shape[2], w.shape[3]
        assert (np.abs(gw[:, :, :cin, :cout] - dw_ref) - 2e-4 * dw_abs).max() <= 1e-30, ("dW", layer)
        assert np.abs(gb[:cout] - db_ref).max() <= 2e-4 * np.abs(dz).sum() / 1 + 1e-12
        # padded channels receive no gradient
        assert np.all(gw[:, :, cin:, :] == 0) and np.all(gw[:, :, :, cout:] == 0)
        assert np.all(gb[cout:] == 0)


def test_adam_matches_oracle(setup):
    net = setup["net"]
    rng = np.random.default_rng(4)
    p = rng.standard_normal(CNN_PARAMS).astype(np.float32)
    g = rng.standard_normal(CNN_PARAMS).astype(np.float32)
    m = (rng.standard_normal(CNN_PARAMS) * 0.1).astype(np.float32)
    v = (rng.random(CNN_PARAMS) * 0.1).astype(np.float32)
    tp, tg, tm, tv = (torch.from_numpy(a).cuda() for a in (p, g, m, v))
    net.adam(tp, tg, tm, tv, 7, lr=1e-3)
    rp, rm, rv = ocl.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                          v.astype(np.float64), 7, lr=1e-3)
    assert np.abs(tp.cpu().numpy() - rp).max() < 1e-6
    assert np.abs(tm.cpu().numpy() - rm).max() < 1e-6
    assert np.abs(tv.cpu().numpy() - rv).max() < 1e-6


def _oracle_lattice():
    import oracle
    return oracle.Lattice(2, N, N, v=[0, 1, -1, 3, -3])


def test_apply_is_the_oracle_equilibrium_shift(setup):
    """apply = equilibrium shift of the streamed correction moments (FP64)."""
    net = setup["net"]
    posts = [p.clone() for p in setup["posts"]]
    net.forward(setup["params"], posts)
    skipped = torch.zeros(1, dtype=torch.int32, device="cuda")
    net.apply(posts, bound=1e30, skipped=skipped)
    assert int(skipped.item()) == 0
    cs = net.activation(7).permute(0, 2, 3, 1).double().cpu().numpy()
    y = np.stack([setup["acts"][3][f][..., :25] for f in range(FRAMES)])
    corr = (y @ ocl.projection(setup["oscale"]).T) * setup["oscale"]
    assert np.abs(cs - corr).max() <= 1e-5 * np.abs(corr).max()
    lat = _oracle_lattice()
    for f in range(FRAMES):
        want = ocl.equilibrium_shift(setup["P"][f], cs[f], lat)
        got = _nodes(posts[f])
        # the shift is computed and kept in FP64
        assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
        # totals of mass, momentum and energy are unchanged up to FP64
        # rounding: each population's shift is the difference of two
        # equilibria, each a few roundings of values of the population's size
        v = ocl.velocities_2d()
        phi = np.stack([np.ones(25), v[:, 0], v[:, 1], (v ** 2).sum(1)], axis=1)
        tot = lambda a: (a.reshape(-1, 25) @ phi).sum(axis=0)
        bound = 1e-14 * (np.abs(got).reshape(-1, 25) @ np.abs(phi)).sum(axis=0)
        assert np.all(np.abs(tot(got) - tot(setup["P"][f])) <= bound)
    # fallback: a bound nothing meets leaves every node unchanged
    posts2 = [p.clone() for p in setup["posts"]]
    net.forward(setup["params"], posts2)
    skipped.zero_()
    net.apply(posts2, bound=1e-12, skipped=skipped)
    assert int(skipped.item()) == FRAMES * N * N
    for a, b in zip(posts2, setup["posts"]):
        assert torch.equal(a, b)


def test_non_finite_network_falls_back_to_the_plain_step(setup):
    """Parameters poisoned with NaN make every correction non-finite: apply
    skips every node and leaves the post buffers bitwise unchanged, so the
    run continues as the plain coarse step."""
    net = setup["net"]
    bad = setup["params"].clone()
    bad[::97] = float("nan")
    posts = [p.clone() for p in setup["posts"]]
    net.forward(bad, posts)
    skipped = torch.zeros(1, dtype=torch.int32, device="cuda")
    net.apply(posts, bound=1e30, skipped=skipped)
    assert int(skipped.item()) == FRAMES * N * N
    for a, b in zip(posts, setup["posts"]):
        assert torch.equal(a, b)
    net.forward(setup["params"], setup["posts"])            # leave the clean activations


def test_fp32_posts_are_read_and_shifted_in_fp32():
    fields = inputs.kelvin_helmholtz(N, N, u0=0.08, delta=3.0, theta=0.35)
    lat = Lattice(2, N, N, omega=1.9, storage="f32").init(*fields)
    lat.step(2)
    net = Closure(N, N, 1, storage="f32")
    P = _nodes(lat.f)[None]
    mean = P.mean(axis=(0, 1, 2))
    scale = P.std(axis=(0, 1, 2)) + 1e-6
    oscale = 1e-3 * mean / mean.sum()
    net.set_norm(mean, scale, oscale, [1.0] * 4)
    params = init_params(seed=4, out_gain=1.0)
    post = lat.f.clone()
    net.forward(params, [post])
    x0 = net.activation(0).double().cpu().numpy()
    X = (P - mean) / scale
    assert np.abs(x0[..., :25] - X).max() <= BF * np.abs(X).max() + 1e-6
    net.apply([post], bound=1e30)
    cs = net.activation(7)[0].permute(1, 2, 0).double().cpu().numpy()
    want = ocl.equilibrium_shift(P[0], cs, _oracle_lattice())
    got = _nodes(post)
    assert np.abs(want - P[0]).max() > 0
    # FP32 storage: the sum is rounded to FP32
    assert np.abs(got - want).max() <= 2.0 ** -24 * np.abs(want).max() * 1.01


def test_restriction_matches_oracle():
    rng = np.random.default_rng(1)
    n = 64
    rho = 1 + 0.05 * rng.standard_normal((n, n))
    ux, uy = 0.05 * rng.standard_normal((2, n, n))
    th = 0.35 + 0.01 * rng.standard_normal((n, n))
    got = restrict(*[torch.from_numpy(a).cuda() for a in (rho, ux, uy, th)])
    ref = ocl.restrict(rho, rho * ux, rho * uy, rho * (2 * th + ux ** 2 + uy ** 2))
    for a, b in zip(got, ref):
        assert np.abs(a.cpu().numpy() - b).max() < 1e-13


def test_training_reduces_loss():
    from paper_1402_5487_amd.closure_train import Experiment
    ex = Experiment(n_coarse=64, factor=4, batch=4)
    ex.generate(seeds=range(4), per_seed=6, horizon=60)
    ex.fit_norm()
    held = ex.frames[-4:]
    ex.frames = ex.frames[:-4]
    hist = ex.train(300, lr=2e-3, log_every=50)
    print("loss history", hist)
    assert np.isfinite(hist[-1][1])
    assert hist[-1][1] < 0.7 * hist[0][1], hist
    assert np.isfinite(ex.loss_on(held))


def test_trained_closure_gains_on_held_out_steps():
    """The one-step training path (Experiment.train on one-step targets, the
    library's plbm_closure_backward): on frames of held-out seeds, the share
    of the one-step error of the conserved densities (against the restricted
    fine run) that the corrected step removes.  This path learns single
    steps but does not improve rollouts; the shipped closure is trained
    through coarse steps and its rollout gain is asserted in
    test_gpu_closure_rollout."""
    from paper_1402_5487_amd.closure_train import Experiment
    ex = Experiment(n_coarse=128, factor=4, batch=8)
    ex.generate(seeds=range(100, 102), per_seed=8, horizon=120, rng_seed=3)
    held = [f for f in ex.frames if f[2] >= 3]
    ex.frames = []
    ex.generate(seeds=range(12), per_seed=10, horizon=120)
    ex.frames = [f for f in ex.frames if f[2] >= 3]
    ex.fit_norm()
    ex.train(800, lr=1e-3)
    l0, l1, gain = ex.explained(held)
    print(f"held-out one-step loss plain {l0:.4g} closure {l1:.4g} explained {gain:.3f}")
    assert np.isfinite(l1)
    assert gain > GAIN_MIN, (l0, l1)
