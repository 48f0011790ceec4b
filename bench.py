"""Throughput of the fused parametric-LBM step on one MI355X.

Workload: D2Q25 thermal Kelvin-Helmholtz double shear layer (tensor product
of D1Q5 {0, +-1, +-3}), 4096 x 4096 periodic nodes, U0 = 0.1, delta = L/80,
u_y = 0.005 sin(2 pi x/L), omega = 1.8.  Temperature theta = 0.35: the stable
variant of the literal theta = 0.3, which is linearly unstable (round-off
grows ~6% per step and FP16 storage goes non-finite within ~200 steps).
Throughput does not depend on the values; the stable variant keeps every
timed step finite.

One step = one fused collide-and-stream launch over all nodes (plbm_step).
The headline is the FP16-deviation storage form (FP32 arithmetic, 100 B per
node per step); the plain FP64 step (400 B), FP32 storage (200 B) and
BF16-deviation storage are timed beside it.  Each form's error is stated
against the FP64 form after --accuracy-steps steps from the same initial
state (the FP64 form matches the CPU oracle to 1e-12 in the test suite).

Prints ONE JSON line (N = 1).
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS and % of HBM roofline, D2Q25 thermal KH 4096², "
          "vs plain FP64 step at stated err")
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = [os.path.join(ROOT, "paper_1402_5487_amd", "csrc", n)
              for n in ("plbm_kernels.hip", "plbm_device.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step2d_kh4096_traffic.json")
COMPUTE_DTYPE = {"f64": "f64", "f32": "f32", "f16dev": "f32", "bf16dev": "f32",
                 "f16dev_sr": "f32", "bf16dev_sr": "f32"}


def kernel_hash():
    """Hash of the step kernel's sources: stored HBM counter totals are used
    only while it matches."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(form, path=TRAFFIC_FILE):
    """HBM bytes per launch of the step in `form` from the stored counter
    totals, or None when they are missing or were taken on other sources."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tr = json.load(fh)
    if tr.get("kernel_sha256_16") != kernel_hash() or form not in tr.get("forms", {}):
        return None
    return tr["forms"][form]["hbm_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--forms", default="f16dev,f64,f32,bf16dev,f16dev_sr,bf16dev_sr")
    ap.add_argument("--theta", type=float, default=0.35)
    ap.add_argument("--accuracy-steps", type=int, default=5000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--only", default=None,
                    help="time one form and print its line only (for profilers)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only the 2 GiB calibration copy (for profilers)")
    ap.add_argument("--batch-steps", type=int, default=2000,
                    help="steps of the batching form (0 skips it)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batching form (for profilers)")
    ap.add_argument("--closure-iters", type=int, default=2000,
                    help="training iterations (segments of 32 coarse steps x 8 runs) of the "
                         "learned closure (0 skips it)")
    ap.add_argument("--closure-storage", default="f32", choices=("f32", "f64"),
                    help="populations of the coarse lattice the closure corrects")
    ap.add_argument("--closure-train-seeds", type=int, default=200)
    ap.add_argument("--closure-held-seeds", type=int, default=20)
    ap.add_argument("--q9-forms", default="q9f64,q9f32",
                    help="D2Q9 isothermal (zeta = 4) forms timed beside the D2Q25 ones "
                         "(empty: none)")
    ap.add_argument("--gen-forms", default="d2q16:f32,d2q49:f32,d2q49:f64",
                    help="general velocity sets (model:storage) timed at the KH size (empty: skip)")
    ap.add_argument("--gen-only", action="store_true",
                    help="time only the general-set forms and print their line")
    ap.add_argument("--d3-forms", default="f64,f32",
                    help="storage forms of the D3Q125 Taylor-Green line (empty: skip)")
    ap.add_argument("--d3-size", type=int, default=256)
    ap.add_argument("--d3-only", action="store_true",
                    help="time only the D3Q125 forms and print their line")
    ap.add_argument("--kh1024-steps", type=int, default=10000,
                    help="steps of the FP32 1024x1024 KH run compared with FP64 (0 skips it)")
    ap.add_argument("--closure-only", action="store_true",
                    help="run only the learned-closure experiment")
    ap.add_argument("--oracle-size", type=int, default=256,
                    help="KH size at which every form is compared with the oracle directly")
    ap.add_argument("--oracle-checkpoints", default="500,1000,2000,3000",
                    help="steps at which they are compared (empty: skip)")
    ap.add_argument("--literal-limit", type=int, default=3000,
                    help="steps the literal theta = 0.3 KH runs at most per form (0 skips)")
    ap.add_argument("--literal-batch-steps", type=int, default=2000,
                    help="steps of the literal-theta batch (0 skips)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_lattice(storage, n, fields, theta):
    """D2Q25 lattice of the given storage, or for "q9f64" / "q9f32" the
    isothermal D2Q9 lattice of the three-velocity family with zeta = 4
    (theta0 = 1/4; the theta field is not used)."""
    from paper_1402_5487_amd.lattice import Lattice
    if storage.startswith("q9"):
        return Lattice(2, n, n, omega=1.8, storage=storage[2:], zeta=4.0).init(*fields)
    if storage.endswith("_sr"):          # 16-bit deviations, stochastic rounding
        return Lattice(2, n, n, omega=1.8, storage=storage[:-3], theta0=theta,
                       rounding="stochastic").init(*fields)
    return Lattice(2, n, n, omega=1.8, storage=storage, theta0=theta).init(*fields)


WINDOWS = 5


def timed_windows(step, steps, windows=WINDOWS):
    """Per-step times (ms) of `windows` back-to-back windows of exactly
    `steps` steps, each bracketed by synchronisation and timed with HIP
    events on the stream the library launches on (torch's current stream,
    handed to every plbm_step call)."""
    import torch
    stream = torch.cuda.current_stream()
    out = []
    for _ in range(windows):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / steps)
    return out


def summarize(times, nodes, bytes_step):
    """Median window and the spread of all windows."""
    ms = statistics.median(times)
    gbs = bytes_step / (ms * 1e-3) / 1e9
    return {"ms_per_step": ms, "mlups": nodes / (ms * 1e-3) / 1e6, "gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS, "bytes_per_node": bytes_step // nodes,
            "windows": len(times), "window_ms": [min(times), max(times)],
            "frac_range": [bytes_step / (max(times) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           bytes_step / (min(times) * 1e-3) / 1e9 / HBM_PEAK_GBS]}


PREWARM_MS = 100.0


def device_prewarm(storage, n, fields, theta, ms=PREWARM_MS):
    """Sustained load before a form is timed: the same form's step on a
    separate lattice of the same size for `ms` milliseconds.  After the idle
    gap of a lattice's initialisation the first 20-60 launches of a 16-bit
    step run 5-25 % slower while the clock settles (traced with rocprofv3);
    a 5000-step job spends under 2 % of its time there, and each form's
    whole 5000-step run is timed as well (`job_5000`).  The timed lattice
    still gets exactly W warm-up steps and K timed steps."""
    import torch
    scratch = make_lattice(storage, n, fields, theta)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    done = 0.0
    while done < ms:
        e0.record(st)
        scratch.step(10)
        e1.record(st)
        e1.synchronize()
        done += e0.elapsed_time(e1)
    # (the scratch buffers go back to torch's cache, not to the driver: no
    # idle gap before the timed lattice starts)
    del scratch


def time_form(storage, n, fields, steps, warmup, theta):
    """Device pre-warm, W warm-up steps, then the median of WINDOWS windows
    of `steps` steps."""
    import torch
    lat = make_lattice(storage, n, fields, theta)
    device_prewarm(storage, n, fields, theta)
    lat.step(warmup)
    times = timed_windows(lat.step, steps)
    out = summarize(times, n * n, lat.bytes_per_step)
    out["finite_after"] = bool(torch.isfinite(lat.moments()[0]).all())
    del lat
    torch.cuda.empty_cache()
    return out


def time_form3(storage, n, fields, steps, warmup):
    """The D3Q125 step (Sec. 2.4) on an n^3 Taylor-Green box, timed like
    time_form."""
    import torch
    from paper_1402_5487_amd.lattice import Lattice3
    lat = Lattice3(n, n, n, omega=1.6, storage=storage).init(*fields)
    lat.step(warmup)
    times = timed_windows(lat.step, steps)
    out = summarize(times, n ** 3, lat.bytes_per_step)
    out["finite_after"] = bool(torch.isfinite(lat.moments()[0]).all())
    del lat
    torch.cuda.empty_cache()
    return out


def d3_forms(args):
    from paper_1402_5487_amd import inputs
    forms = [f for f in args.d3_forms.split(",") if f]
    if not forms:
        return None
    n = args.d3_size
    fields = inputs.taylor_green_3d(n, n, n, u0=0.05, theta=1.0 / 3.0)
    out = {"workload": f"D3Q125 Taylor-Green {n}^3 periodic, u0=0.05, omega=1.6"}
    steps = max(1, args.steps // 4)
    for storage in forms:
        log(f"timing d3q125 {storage} {n}^3 steps={steps} warmup={args.warmup}")
        out[storage] = time_form3(storage, n, fields, steps, args.warmup)
    return out


# general on-lattice sets (Sec. 2.2) run through the general kernels:
# (velocities, temperature, isothermal)
GEN_SETS = {"d2q16": ((1, -1, 3, -3), 4.0 / 3.0, True),
            "d2q49": ((0, 1, -1, 2, -2, 3, -3), 1.0, False)}


def time_gen(model, storage, n, steps, warmup):
    """A general-set lattice on the KH workload at its own temperature, timed
    like time_form."""
    import torch
    from paper_1402_5487_amd import inputs
    from paper_1402_5487_amd.lattice import Lattice
    v, th, iso = GEN_SETS[model]
    lat = Lattice(2, n, n, omega=1.8, storage=storage, velocities=v, theta0=th if iso else None)
    lat.init(*inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80.0, theta=th))
    lat.step(warmup)
    times = timed_windows(lat.step, steps)
    out = {"velocities": list(v), "theta": th, "isothermal": iso,
           **summarize(times, n * n, lat.bytes_per_step)}
    out["finite_after"] = bool(torch.isfinite(lat.moments()[0]).all())
    del lat
    torch.cuda.empty_cache()
    return out


def gen_forms(args):
    forms = [f for f in args.gen_forms.split(",") if f]
    if not forms:
        return None
    out = {"workload": f"KH {args.size}x{args.size} periodic, u0=0.1, omega=1.8, "
                       "each set at its own temperature"}
    for form in forms:
        model, storage = form.split(":")
        log(f"timing general {model} {storage} {args.size}^2 steps={args.steps}")
        out[form] = time_gen(model, storage, args.size, args.steps, args.warmup)
    return out


def accuracy(forms, n, fields, steps, theta):
    """Max abs error of rho, u, theta against the FP64 form after `steps`,
    and the normwise relative errors ||m - m_ref||_2 / ||m_ref||_2."""
    import torch
    out, jobs = {}, {}
    ref = None
    for storage in ["f64"] + [f for f in forms if f != "f64"]:
        log(f"accuracy {storage} {steps} steps")
        lat = make_lattice(storage, n, fields, theta)
        job_ms = timed_windows(lat.step, steps, windows=1)[0] * steps
        job = {"steps": steps, "ms": job_ms,
               "mlups": n * n * steps / (job_ms * 1e-3) / 1e6,
               "frac": lat.bytes_per_step * steps / (job_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        mom = [t for t in lat.moments()]
        del lat
        torch.cuda.empty_cache()
        jobs[storage] = job
        if ref is None:
            ref = mom
            continue
        out[storage] = {"steps": steps,
                        "rho": float((mom[0] - ref[0]).abs().max()),
                        "ux": float((mom[1] - ref[1]).abs().max()),
                        "uy": float((mom[2] - ref[2]).abs().max()),
                        "theta": float((mom[3] - ref[3]).abs().max()),
                        "rel_l2": {k: float((a - b).norm() / b.norm())
                                   for k, a, b in zip(("rho", "ux", "uy", "theta"), mom, ref)},
                        "finite": bool(torch.isfinite(mom[0]).all())}
        del mom
    return out, jobs


def kh1024_form(args):
    """The FP32 KH configuration at 1024^2 (delta = 12.8, theta = 0.35,
    omega = 1.8): step rate, and the max abs error of rho, u, theta against
    the FP64 run after --kh1024-steps steps."""
    from paper_1402_5487_amd import inputs
    n = 1024
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80.0, theta=args.theta)
    log(f"timing f32 {n}x{n} steps={args.steps} warmup={args.warmup}")
    out = {"workload": f"D2Q25 thermal KH {n}x{n} periodic, FP32, theta={args.theta}, omega=1.8",
           "note": "the two buffers (210 MB) fit the 256 MB Infinity Cache: not an HBM "
                   "measurement; the rate is against 8 TB/s only for comparison"}
    out["f32"] = time_form("f32", n, fields, args.steps, args.warmup, args.theta)
    errs, jobs = accuracy(["f32"], n, fields, args.kh1024_steps, args.theta)
    out["f32"]["max_abs_err_vs_fp64_ref"] = errs["f32"]
    out["f32"]["job_%d" % args.kh1024_steps] = jobs["f32"]
    return out


def transport_errors():
    """Relative errors of the viscosity (decaying shear wave, 128^2, u = 0.01,
    400 steps) and of the thermal diffusivity (isobaric entropy wave, 128 x 8,
    1200 steps) against nu = (1/omega - 1/2) theta, per storage form, omega = 1."""
    import numpy as np
    from paper_1402_5487_amd import inputs
    from paper_1402_5487_amd.lattice import Lattice

    def lat(nx, ny, form, th0):
        st, rnd = (form[:-3], "stochastic") if form.endswith("_sr") else (form, "nearest")
        return Lattice(2, nx, ny, omega=1.0, storage=st, theta0=th0, rounding=rnd)

    out = {}
    for form in ("f64", "f32", "f16dev", "bf16dev", "f16dev_sr", "bf16dev_sr"):
        L, th = 128, 0.35
        a = lat(L, L, form, th).init(*inputs.shear_wave(L, L, amp=0.01, theta=th))
        s = np.sin(2 * np.pi * np.arange(L) / L)
        amp = lambda: (a.moments()[1].cpu().numpy().mean(axis=1) * s).sum() / (s * s).sum()
        a0 = amp()
        a.step(400)
        k = 2 * np.pi / L
        e_nu = -np.log(amp() / a0) / (k * k * 400) / (0.5 * th) - 1
        th0, x = 0.5, np.arange(L)
        tt = np.tile(th0 * (1 + 0.01 * np.sin(2 * np.pi * x / L)), (8, 1))
        rho = th0 / tt
        b = lat(L, 8, form, th0).init(rho, 0 * rho, 0 * rho, tt)

        def ent():
            m = [t.cpu().numpy() for t in b.moments()]
            return ((m[3].mean(axis=0) - th0) / th0 - (m[0].mean(axis=0) - 1)) @ np.sin(2 * np.pi * x / L)
        b0 = ent()
        b.step(1200)
        e_k = -np.log(ent() / b0) / (k * k * 1200) / (0.5 * th0) - 1
        out[form] = {"nu_rel_err": float(e_nu), "thermal_diffusivity_rel_err": float(e_k)}
    return out


def copy_bandwidth(reps=20):
    """plbm_stream_copy of 2 GiB: the achievable HBM rate on this machine."""
    import torch
    from paper_1402_5487_amd import _plbm
    nbytes = 1 << 31
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(3):
        _plbm.stream_copy(a, b, nbytes, st.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        _plbm.stream_copy(a, b, nbytes, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / reps * 1e-3
    ok = bool(torch.equal(a[:1024], b[:1024]))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / s / 1e9, ok


def batch_form(steps, seed=0):
    """256 independent KH lattices, sides drawn from {64, 96, ..., 512},
    U0 ~ U[0.02, 0.12], theta ~ U[0.345, 0.355] (stable variant of
    U[0.2, 0.4]), omega ~ U[1.5, 1.9]; autotuned tiles, one launch per step
    replayed from a captured graph.  The 2000 steps of each lattice are
    timed as the median of WINDOWS windows of steps / WINDOWS launches."""
    import tempfile

    import torch
    from paper_1402_5487_amd import inputs
    from paper_1402_5487_amd.batch import Batch
    members = inputs.batch_members(256, seed=seed, theta_range=(0.345, 0.355))
    b = Batch([(m.side, m.side, m.omega) for m in members])
    t0 = time.perf_counter()
    with tempfile.TemporaryDirectory() as td:
        b.autotune(os.path.join(td, "tune.json"))
    tune_s = time.perf_counter() - t0
    for i, m in enumerate(members):
        b.init(i, *inputs.kelvin_helmholtz(m.side, m.side, u0=m.u0, theta=m.theta))
    b.step(16)                                     # warm-up, records the graph
    per = max(8, (steps // WINDOWS) // 8 * 8)      # whole graphs of 8 launches
    times = timed_windows(b.step, per)
    info = b.info()
    finite = all(bool(torch.isfinite(b.moments(i)[0]).all()) for i in range(0, 256, 17))
    b.close()
    nodes = info["nodes"]
    out = {"lattices": 256, "nodes": nodes, "steps": per * WINDOWS,
           **summarize(times, nodes, nodes * 200)}
    out.update({"tiles": info["tiles"], "grid_mode": info["grid_mode"],
                "lds_bytes": info["lds_bytes"], "graph_steps": info["graph_steps"],
                "tile_shapes": {str(k): list(v) for k, v in sorted(info["classes"].items())},
                "autotune_s": tune_s, "finite_sampled": finite})
    return out


def predicted_growth(members, nk=24):
    """Largest von Neumann amplification per step of the D2Q25 SRT update
    around uniform states at each (theta, u0, omega) of `members` (flow
    (u0, 0) and rest), from the oracle's own Jacobian (oracle/stability.py).
    Part of the CPU (oracle) leg."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from oracle import stability

    def one(m):
        theta, u0, omega = m
        lat = oracle.Lattice(2, 1, 1, omega=omega)
        return max(stability.max_amplification(lat, 1.0, u0, 0.0, theta, nk=nk),
                   stability.max_amplification(lat, 1.0, 0.0, 0.0, theta, nk=nk))
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        return list(ex.map(one, members))


def first_nonfinite(step_sums, limit, every):
    """Step count at which the fused FP64 sums first report a non-finite
    state (checked every `every` steps), or None if still finite at limit."""
    from paper_1402_5487_amd import _plbm
    t = 0
    while t < limit:
        try:
            step_sums(every)
        except _plbm.PlbmError as e:
            if e.status != _plbm.PLBM_ENONFINITE:
                raise
            return t + every
        t += every
    return None


# relative size of one store's rounding: the unit roundoff for FP64 and FP32;
# for the 16-bit forms half an ulp of a deviation of a few per cent of the
# population
STORE_NOISE = {"f64": 1.1e-16, "f32": 6e-8, "f16dev": 2e-5, "bf16dev": 2e-4}


def literal_kh(n, forms, limit=3000, every=25):
    """The literal configuration theta = 0.3 (linearly unstable at
    omega = 1.8): first non-finite step per storage form (the CPU leg adds
    the von Neumann prediction)."""
    import torch
    from paper_1402_5487_amd import inputs
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80.0, theta=0.3)
    out = {"workload": f"D2Q25 KH {n}x{n}, theta=0.3 (literal), omega=1.8, u0=0.1",
           "checked_every": every, "limit": limit}
    for form in forms:
        lat = make_lattice(form, n, fields, 0.3)
        step = first_nonfinite(lambda k: lat.step(k, sums=True), limit, every)
        out[form] = {"first_nonfinite_step": step}
        log(f"literal KH {form}: non-finite at {step}")
        del lat
        torch.cuda.empty_cache()
    return out


def predict_literal_kh(lit):
    """Growth factor of the literal KH state and the step at which each
    form's store rounding would reach order one growing at that rate."""
    import math
    lam = predicted_growth([(0.3, 0.1, 1.8)], nk=48)[0]
    lit["growth_per_step"] = lam
    for form, v in lit.items():
        if isinstance(v, dict) and "first_nonfinite_step" in v:
            base = form[:-3] if form.endswith("_sr") else form
            v["predicted_step"] = math.log(1.0 / STORE_NOISE[base]) / math.log(lam) \
                if lam > 1 else None


def literal_batch(steps, seed=0, every=50):
    """The literal batch, theta ~ U[0.2, 0.4] (same seed, so the same sides,
    U0 and omega as the stable variant): which lattices go non-finite and
    when (the CPU leg adds each lattice's von Neumann growth)."""
    from paper_1402_5487_amd import _plbm, inputs
    from paper_1402_5487_amd.batch import Batch
    members = inputs.batch_members(256, seed=seed)
    b = Batch([(m.side, m.side, m.omega) for m in members])
    for i, m in enumerate(members):
        b.init(i, *inputs.kelvin_helmholtz(m.side, m.side, u0=m.u0, theta=m.theta))
    first = [None] * len(members)
    t = 0
    while t < steps:
        b.step(every)
        t += every
        for i in range(len(members)):
            if first[i] is not None:
                continue
            try:
                b.moments(i, sums=True)
            except _plbm.PlbmError as e:
                if e.status != _plbm.PLBM_ENONFINITE:
                    raise
                first[i] = t
    b.close()
    blew = [i for i, s in enumerate(first) if s is not None]
    return {"workload": "256 D2Q25 KH lattices, sides {64..512}, theta ~ U[0.2, 0.4] (literal), "
                        "U0 ~ U[0.02, 0.12], omega ~ U[1.5, 1.9], FP32",
            "steps": steps, "checked_every": every, "nonfinite": len(blew),
            "first_nonfinite_steps": sorted(s for s in first if s is not None),
            "theta_max_nonfinite": max((members[i].theta for i in blew), default=None),
            "theta_min_finite": min((members[i].theta for i in range(len(members))
                                     if first[i] is None), default=None),
            "_members": [(m.theta, m.u0, m.omega) for m in members], "_first": first}


def predict_literal_batch(lb):
    """Von Neumann growth of every literal-batch lattice; a lattice counts as
    predicted to go non-finite within the run when FP32 rounding (2^-24)
    growing at that rate reaches order one before the last step.  Agreement
    is counted lattice by lattice."""
    import math
    members, first = lb.pop("_members"), lb.pop("_first")
    lam = predicted_growth(members)
    steps = lb["steps"]
    pred = [math.log(2.0 ** 24) / math.log(g) if g > 1 + 1e-9 else None for g in lam]
    within = [p is not None and p < steps for p in pred]
    blew = [f is not None for f in first]
    lb["predicted_unstable"] = sum(p is not None for p in pred)
    lb["predicted_within_steps"] = sum(within)
    lb["agree_with_prediction"] = sum(w == b for w, b in zip(within, blew))
    ratios = [f / p for f, p in zip(first, pred) if f is not None and p is not None]
    lb["observed_over_predicted_step"] = ([min(ratios), statistics.median(ratios), max(ratios)]
                                          if ratios else None)


def closure_form(args):
    """Learned closure: coarse 256^2 KH (FP32 populations, omega viscosity-
    matched), the network trained through coarse steps on the restricted
    1024^2 runs of the training seeds, judged on held-out seeds against the
    restricted fine run over 500 coarse steps (and judged again with FP64
    coarse populations)."""
    from paper_1402_5487_amd import closure_train
    nt, nh = args.closure_train_seeds, args.closure_held_seeds
    return closure_train.run(train_seeds=range(nt), held_seeds=range(200, 200 + nh),
                             iters=args.closure_iters, storage=args.closure_storage, log=log)


def cpu_baseline(n, fields, steps):
    """The FP64 C oracle on the headline lattice: `steps` steps on every host
    thread it is given, and one step on one thread.  Returns the baseline
    entry and the oracle's moments after the `steps` steps (the anchor of the
    GPU's FP64 reference at this size)."""
    import oracle
    lat = oracle.Lattice(2, n, n, omega=1.8)
    f0 = lat.init(*fields)
    threads = oracle.num_threads()
    t = time.perf_counter()
    f = lat.step(f0, steps)
    dt = time.perf_counter() - t
    oracle.set_num_threads(1)
    try:
        t = time.perf_counter()
        lat.step(f0, 1)
        dt1 = time.perf_counter() - t
    finally:
        oracle.set_num_threads(threads)
    return {"value": round(n * n * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "one_thread_mlups": round(n * n / dt1 / 1e6, 3),
            "sample": f"{steps} steps of the same {n}x{n} KH lattice by the FP64 C "
                      f"oracle (OpenMP, {threads} threads), {dt:.1f} s; one step on one "
                      f"thread, {dt1:.1f} s"}, lat.moments(f)


def fp64_anchor(n, fields, steps, theta, ref):
    """Largest relative field difference between the GPU FP64 step and the
    oracle's moments `ref` after the same steps (velocities relative to
    U0 = 0.1 at least)."""
    import torch
    g = make_lattice("f64", n, fields, theta)
    g.step(steps)
    got = [a.cpu().numpy() for a in g.moments()]
    del g
    torch.cuda.empty_cache()
    err = max(float(abs(a - b).max() / max(abs(b).max(), fl))
              for a, b, fl in zip(got, ref, (1.0, 0.1, 0.1, 1.0)))
    return {"size": n, "steps": steps, "max_rel_field_err": err}


def kh_vs_oracle(forms, n, theta, checkpoints):
    """Every storage form against the FP64 oracle on the KH problem at n^2
    (delta = n/80), at each checkpoint, next to the oracle's own
    self-divergence (the same oracle with each node's populations summed in
    reversed order): past the parity horizon no two correct FP64 runs agree
    better than that floor."""
    import oracle
    import torch
    from paper_1402_5487_amd import inputs
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80.0, theta=theta)
    lat = oracle.Lattice(2, n, n, omega=1.8)
    a = b = lat.init(*fields)
    gpu = {f: make_lattice(f, n, fields, theta) for f in forms}
    out = {"workload": f"D2Q25 KH {n}x{n}, theta={theta}, omega=1.8, delta={n / 80.0}",
           "checkpoints": {}}
    t = 0
    for c in checkpoints:
        a = lat.step(a, c - t)
        b = lat.step(b, c - t, reverse_sums=True)
        ref = lat.moments(a)
        rows = {"oracle_self_divergence": _max_abs(lat.moments(b, reverse_sums=True), ref)}
        for f, g in gpu.items():
            g.step(c - t)
            rows[f] = _max_abs([x.cpu().numpy() for x in g.moments()], ref)
        t = c
        out["checkpoints"][str(c)] = rows
        log(f"kh{n} vs oracle at {c}: floor {rows['oracle_self_divergence']['max']:.2e}, "
            + ", ".join(f"{f} {rows[f]['max']:.2e}" for f in forms))
    del gpu
    torch.cuda.empty_cache()
    return out


def _max_abs(got, ref):
    d = {name: float(abs(x - y).max()) for name, x, y in zip(("rho", "ux", "uy", "theta"), got, ref)}
    d["max"] = max(d.values())
    return d


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: libplbm runs on exactly one GPU; the multi-GPU "
              "(y-slab halo exchange) path is design-only, so --gpus N>1 is not "
              "measured.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1402_5487_amd import inputs

    if args.calibrate_copy:
        gbs, ok = copy_bandwidth(reps=10)
        print(json.dumps({"copy_gbs": round(gbs, 1), "ok": ok}), flush=True)
        return

    if args.batch_only:
        print(json.dumps(batch_form(args.batch_steps)), flush=True)
        return
    if args.closure_only:
        print(json.dumps(closure_form(args)), flush=True)
        return
    if args.d3_only:
        print(json.dumps(d3_forms(args)), flush=True)
        return
    if args.gen_only:
        print(json.dumps(gen_forms(args)), flush=True)
        return

    n = args.size
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80.0, theta=args.theta)
    forms = args.forms.split(",") if args.only is None else [args.only]
    copy_gbs, copy_ok = (None, None) if args.only else copy_bandwidth()
    results = {}
    for storage in forms:
        log(f"timing {storage} {n}x{n} steps={args.steps} warmup={args.warmup} x{WINDOWS} windows")
        results[storage] = time_form(storage, n, fields, args.steps, args.warmup, args.theta)
    if args.only is not None:
        print(json.dumps({"form": args.only, **results[args.only]}), flush=True)
        return

    d2q9 = {}
    for storage in [f for f in args.q9_forms.split(",") if f]:
        log(f"timing {storage} {n}x{n} steps={args.steps} warmup={args.warmup}")
        d2q9[storage] = time_form(storage, n, fields, args.steps, args.warmup, args.theta)

    d3 = d3_forms(args)
    gen = gen_forms(args)
    kh1024 = kh1024_form(args) if args.kh1024_steps > 0 else None

    acc, jobs = accuracy(forms, n, fields, args.accuracy_steps, args.theta) \
        if args.accuracy_steps > 0 else ({}, {})
    for k, v in acc.items():
        results[k]["max_abs_err_vs_fp64_ref"] = v
    for k, v in jobs.items():
        results[k]["job_%d" % args.accuracy_steps] = v
    literal = lbatch = None
    if args.literal_limit > 0:
        log("literal theta = 0.3 KH, per storage form")
        literal = literal_kh(n, forms, limit=args.literal_limit)
    if args.literal_batch_steps > 0:
        log("literal batch, theta ~ U[0.2, 0.4]")
        lbatch = literal_batch(args.literal_batch_steps)
    transport = transport_errors()
    batch = None
    if args.batch_steps > 0:
        log(f"batching form, {args.batch_steps} steps")
        batch = batch_form(args.batch_steps)
    closure = None
    if args.closure_iters > 0:
        log("learned closure")
        closure = closure_form(args)

    head = "f16dev" if "f16dev" in results else forms[0]
    h = results[head]
    traffic = stored_traffic(head)
    # the CPU leg: everything that runs the oracle (baseline timing, the
    # anchor of the FP64 reference, the forms against the oracle, and the
    # von Neumann predictions of the literal runs)
    cpu = anchor = small = None
    if not args.no_cpu:
        log("cpu oracle baseline")
        cpu, ref = cpu_baseline(n, fields, args.cpu_steps)
        anchor = fp64_anchor(n, fields, args.cpu_steps, args.theta, ref)
        del ref
        if args.oracle_checkpoints:
            cps = [int(c) for c in args.oracle_checkpoints.split(",")]
            log(f"forms against the oracle at {args.oracle_size}^2, checkpoints {cps}")
            small = kh_vs_oracle(forms, args.oracle_size, args.theta, cps)
        if literal:
            predict_literal_kh(literal)
        if lbatch:
            predict_literal_batch(lbatch)
    if lbatch:
        lbatch.pop("_members", None)
        lbatch.pop("_first", None)

    def rnd(d):
        if isinstance(d, dict):
            return {k: rnd(v) for k, v in d.items()}
        if isinstance(d, list):
            return [rnd(v) for v in d]
        if isinstance(d, float):
            return float(f"{d:.6g}")
        return d

    line = {
        "metric": METRIC,
        "value": round(h["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": COMPUTE_DTYPE[head],
        "data": "synthetic",
        "config": {"workload": f"D2Q25 thermal KH {n}x{n} periodic, {head} storage "
                               f"(FP32 arithmetic), theta={args.theta} stable variant",
                   "nx": n, "ny": n, "storage": head, "theta": args.theta,
                   "omega": 1.8, "u0": 0.1, "delta": n / 80.0,
                   "timing": f"median of {WINDOWS} windows of {args.steps} steps, after "
                             f"{args.warmup} warm-up steps and a {PREWARM_MS:.0f} ms device "
                             f"pre-warm (the same form on a separate lattice); each form's "
                             f"whole {args.accuracy_steps}-step run is timed too "
                             f"(forms.*.job_{args.accuracy_steps})"},
        "roofline": {"bound": "hbm", "achieved": round(h["gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(h["frac"], 4), "traffic": traffic},
        "cpu_baseline": cpu,
        "forms": rnd(results),
        "fp64_ref": rnd({
            "what": "errors of the forms are stated against the GPU FP64 run of the same "
                    "lattice, which is tied to the FP64 oracle: equal to it at this size "
                    "after the oracle's baseline steps (vs_oracle, measured here), to 1e-12 "
                    "on 1024^2 KH for the 2000-step parity horizon and within 10x of the "
                    "oracle's self-divergence past it (GPU parity tests); forms_vs_oracle "
                    "compares every form with the oracle directly at a size it can run",
            "vs_oracle": anchor}),
        "forms_vs_oracle": rnd(small) if small else None,
        "literal_kh": rnd(literal) if literal else None,
        "literal_batch": rnd(lbatch) if lbatch else None,
        "transport": rnd(transport),
        "vs_fp64_speedup": round(h["mlups"] / results["f64"]["mlups"], 3)
        if "f64" in results else None,
        "d2q9": rnd(d2q9) if d2q9 else None,
        "kh1024": rnd(kh1024) if kh1024 else None,
        "d3q125": rnd(d3) if d3 else None,
        "general_sets": rnd(gen) if gen else None,
        "batch": rnd(batch) if batch else None,
        "closure": rnd(closure) if closure else None,
        "copy_gbs": round(copy_gbs, 1),
        "copy_ok": copy_ok,
        "kernel_sha256_16": kernel_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
