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
