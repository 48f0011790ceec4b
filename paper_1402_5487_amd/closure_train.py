"""Training and judging the learned closure with data the method generates.

Host orchestration only: every numerical step is a libplbm call (fine and
coarse steps, moments, restriction, network forward/backward, Adam, apply).

Setting (lattice units, acoustic scaling): a fine D2Q25 lattice of
factor * n nodes per side and a coarse one of n, both with the same velocity
set, so one coarse step spans `factor` fine steps.  The coarse relaxation
constant matches the fine viscosity: (1/omega_c - 1/2) = (1/omega_f - 1/2) /
factor (nu = (1/omega - 1/2) theta dt, Sec. 2.1).

Frames (teacher forcing): R_t are the restricted fine fields at coarse time t
(block means of rho, rho u, E).  The coarse post-collision buffer of the
equilibrium of R_t is the network input; the buffer whose streaming yields
the equilibrium of R_(t+1) is the target.  The network learns the projected
difference (it cannot change mass, momentum or energy of a node).

Judge: on held-out seeds, relative L2 errors of the coarse (rho, u, theta)
against R_t at matched times, plain coarse step versus corrected step.
"""
import math
import random

import torch

from . import inputs
from .closure import Closure, init_params, restrict
from .lattice import Lattice


def coarse_omega(omega_f, factor):
    return 1.0 / (0.5 + (1.0 / omega_f - 0.5) / factor)


class Experiment:
    def __init__(self, n_coarse=256, factor=4, theta=0.35, omega_f=1.8, device="cuda:0",
                 batch=8):
        self.nc, self.factor = n_coarse, factor
        self.nf = n_coarse * factor
        self.theta, self.omega_f = theta, omega_f
        self.omega_c = coarse_omega(omega_f, factor)
        self.device = torch.device(device)
        self.batch = batch
        self.net = Closure(self.nc, self.nc, batch, device)
        self.frames = []          # (post, target) FP32 coarse buffers
        self.params = None

    # -- data ------------------------------------------------------------
    def fine_fields(self, seed):
        s = inputs.closure_seed(seed)
        return inputs.kelvin_helmholtz(self.nf, self.nf, u0=s.u0, delta=self.nf / 80.0,
                                       theta=self.theta, uy_amp=s.uy_amp, mode=s.mode,
                                       phase=s.phase)

    def restricted_run(self, seed, times):
        """Restricted fine fields at the coarse times in `times` (sorted)."""
        fine = Lattice(2, self.nf, self.nf, omega=self.omega_f, storage="f32",
                       device=self.device).init(*self.fine_fields(seed))
        out, t = {}, 0
        for want in sorted(set(times)):
            fine.step((want - t) * self.factor)
            t = want
            rho, ux, uy, th = fine.moments()
            out[want] = restrict(rho, ux, uy, th, self.factor)
        return out

    def coarse_lattice(self):
        return Lattice(2, self.nc, self.nc, omega=self.omega_c, storage="f32", device=self.device)

    def make_frame(self, r_t, r_t1):
        lat = self.coarse_lattice().init(*r_t)
        lat.step(1)                       # post-collision of the equilibrium of R_t
        post = lat.f.clone()
        tgt = self.coarse_lattice().init(*r_t1)
        return post, tgt.f.clone()

    def generate(self, seeds, per_seed, horizon, rng_seed=0):
        rng = random.Random(rng_seed)
        for seed in seeds:
            ts = sorted(rng.sample(range(horizon), per_seed))
            fields = self.restricted_run(seed, ts + [t + 1 for t in ts])
            for t in ts:
                self.frames.append(self.make_frame(fields[t], fields[t + 1]))

    # -- normalisation ---------------------------------------------------
    def fit_norm(self, sample=16):
        """Per-population mean/scale of the inputs and scale of the targets
        (setup statistics over a sample of frames)."""
        nc = self.nc
        ps = torch.stack([p.view(nc, 25, nc) for p, _ in self.frames[:sample]])
        ds = torch.stack([(t - p).view(nc, 25, nc) for p, t in self.frames[:sample]])
        mean = ps.mean(dim=(0, 1, 3))
        scale = ps.std(dim=(0, 1, 3)).clamp_min(1e-12)
        oscale = ds.std(dim=(0, 1, 3)).clamp_min(1e-12)
        self.norm = (mean.tolist(), scale.tolist(), oscale.tolist())
        self.net.set_norm(*self.norm)

    # -- training --------------------------------------------------------
    def train(self, iters, lr=1e-3, seed=0, log_every=0):
        if self.params is None:
            self.params = init_params(seed, self.device)
        p = self.params
        g = torch.zeros_like(p)
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        rng = random.Random(seed)
        hist = []
        for it in range(1, iters + 1):
            idx = [rng.randrange(len(self.frames)) for _ in range(self.batch)]
            posts = [self.frames[i][0] for i in idx]
            tgts = [self.frames[i][1] for i in idx]
            self.net.forward(p, posts)
            want = log_every and (it % log_every == 0 or it == 1)
            loss = self.net.backward(p, posts, tgts, g, want_loss=bool(want))
            self.net.adam(p, g, m, v, it, lr=lr * min(1.0, it / 50.0))
            if want:
                hist.append((it, loss))
        torch.cuda.synchronize(self.device)
        return hist

    def loss_on(self, frames):
        g = torch.zeros_like(self.params)
        tot = 0.0
        for i in range(0, len(frames) - self.batch + 1, self.batch):
            posts = [f[0] for f in frames[i:i + self.batch]]
            tgts = [f[1] for f in frames[i:i + self.batch]]
            self.net.forward(self.params, posts)
            tot += self.net.backward(self.params, posts, tgts, g, want_loss=True)
        return tot / max(1, len(frames) // self.batch)

    # -- judging ---------------------------------------------------------
    def judge(self, seed, steps, every, bound=8.0):
        """Relative L2 errors (rho, |u|, theta) of plain and corrected coarse
        runs against the restricted fine run, averaged over t = every,
        2 every, ..., steps."""
        times = list(range(0, steps + 1, every))
        ref = self.restricted_run(seed, times)
        plain = self.coarse_lattice().init(*ref[0])
        corr = self.coarse_lattice().init(*ref[0])
        skipped = torch.zeros(1, dtype=torch.int32, device=self.device)
        err = {"plain": [0.0, 0.0, 0.0], "closure": [0.0, 0.0, 0.0]}
        t = 0
        for want in times[1:]:
            plain.step(want - t)
            for _ in range(want - t):
                corr.step(1)
                self.net.forward(self.params, [corr.f])
                self.net.apply([corr.f], bound=bound, skipped=skipped)
            t = want
            r = ref[want]
            for name, lat in (("plain", plain), ("closure", corr)):
                m = lat.moments()
                e = err[name]
                e[0] += float((m[0] - r[0]).norm() / r[0].norm())
                du = torch.sqrt((m[1] - r[1]) ** 2 + (m[2] - r[2]) ** 2).norm()
                e[1] += float(du / torch.sqrt(r[1] ** 2 + r[2] ** 2).norm())
                e[2] += float((m[3] - r[3]).norm() / r[3].norm())
        k = len(times) - 1
        out = {name: [x / k for x in e] for name, e in err.items()}
        out["skipped_nodes"] = int(skipped.item())
        finite = all(math.isfinite(x) for x in out["closure"])
        out["finite"] = finite
        return out


def forward_rate(ex, reps=20):
    """Inference throughput of the network on one batch: algorithmic FLOPs
    (2 * 9 * (25*32 + 32*32 + 32*25) per node) over the measured time."""
    posts = [f[0] for f in ex.frames[:ex.batch]]
    ex.net.forward(ex.params, posts)
    torch.cuda.synchronize(ex.device)
    st = torch.cuda.current_stream(ex.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        ex.net.forward(ex.params, posts)
    e1.record(st)
    torch.cuda.synchronize(ex.device)
    ms = e0.elapsed_time(e1) / reps
    nodes = ex.batch * ex.nc * ex.nc
    flops = 2 * 9 * (25 * 32 + 32 * 32 + 32 * 25) * nodes
    return ms, flops / (ms * 1e-3) / 1e12


def run(n_coarse=256, factor=4, train_seeds=range(200), held_seeds=range(200, 220),
        per_seed=10, horizon=500, iters=2000, batch=8, lr=1e-3, judge_steps=500,
        judge_every=50, log=None):
    """The full learned-closure experiment: generate, train, judge."""
    import time
    say = log or (lambda msg: None)
    ex = Experiment(n_coarse=n_coarse, factor=factor, batch=batch)
    t0 = time.perf_counter()
    ex.generate(train_seeds, per_seed, horizon)
    gen_s = time.perf_counter() - t0
    say(f"closure: {len(ex.frames)} frames in {gen_s:.1f} s")
    ex.fit_norm()
    t0 = time.perf_counter()
    hist = ex.train(iters, lr=lr, log_every=max(1, iters // 10))
    train_s = time.perf_counter() - t0
    say(f"closure: trained {iters} iterations in {train_s:.1f} s, loss {hist[0][1]:.4g} -> {hist[-1][1]:.4g}")
    fwd_ms, fwd_tflops = forward_rate(ex)
    judged = []
    for s in held_seeds:
        judged.append(ex.judge(s, judge_steps, judge_every))
    plain = [sum(j["plain"][i] for j in judged) / len(judged) for i in range(3)]
    corr = [sum(j["closure"][i] for j in judged) / len(judged) for i in range(3)]
    return {"coarse": n_coarse, "fine": n_coarse * factor, "omega_c": ex.omega_c,
            "train_seeds": len(list(train_seeds)), "held_out_seeds": len(judged),
            "frames": len(ex.frames), "iters": iters, "batch": batch,
            "loss_first": hist[0][1], "loss_last": hist[-1][1], "gen_s": gen_s,
            "train_s": train_s, "ms_per_iter": 1e3 * train_s / iters,
            "forward_ms_per_batch": fwd_ms, "forward_tflops": fwd_tflops,
            "judge_steps": judge_steps,
            "rel_l2_plain": {"rho": plain[0], "u": plain[1], "theta": plain[2]},
            "rel_l2_closure": {"rho": corr[0], "u": corr[1], "theta": corr[2]},
            "gain": {"rho": plain[0] / corr[0], "u": plain[1] / corr[1],
                     "theta": plain[2] / corr[2]},
            "skipped_nodes": sum(j["skipped_nodes"] for j in judged),
            "finite": all(j["finite"] for j in judged)}
