"""Throughput of the fused parametric-LBM step on one MI355X.

Workload: D2Q25 thermal Kelvin-Helmholtz double shear layer, 4096 x 4096
periodic nodes, U0 = 0.1, delta = L/80, u_y = 0.005 sin(2 pi x/L), theta = 0.3,
omega = 1.8 (the literal parameters; throughput does not depend on the values).
One "step" is one fused collide-and-stream pass over all nodes
(one plbm_step launch).  The headline is the 16-bit (FP16) deviation-storage
form with FP32 arithmetic; the plain FP64, FP32 and BF16-deviation forms are
timed beside it, each with its error against the FP64 form after the same
steps (the FP64 form itself is checked against the CPU oracle at 1e-12 by the
test suite).

Prints ONE JSON line (rank 0, N = 1).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS and % of HBM roofline, D2Q25 thermal KH 4096², "
          "vs plain FP64 step at stated err")
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1402_5487_amd", "csrc", "plbm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step2d_kh4096_traffic.json")


def kernel_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--forms", default="f16dev,f64,f32,bf16dev")
    ap.add_argument("--theta", type=float, default=0.3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--only", default=None,
                    help="time a single form and print nothing else (profiling)")
    return ap.parse_args()


def time_form(storage, n, fields, steps, warmup, theta):
    import torch
    from paper_1402_5487_amd.lattice import Lattice
    lat = Lattice(2, n, n, omega=1.8, storage=storage, theta0=theta)
    lat.init(*fields)
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall = time.perf_counter()
    t0.record(stream)
    lat.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    ms = t0.elapsed_time(t1) / steps
    mlups = n * n / (ms * 1e-3) / 1e6
    gbs = lat.bytes_per_step / (ms * 1e-3) / 1e9
    mom = [t.double() for t in lat.moments()]
    return lat, {"ms_per_step": ms, "mlups": mlups, "gbs": gbs,
                 "frac": gbs / HBM_PEAK_GBS, "bytes_per_node": lat.bytes_per_step // (n * n),
                 "wall_s": wall}, mom


def copy_bandwidth():
    """Plain device copy of 2 GiB (read + write), the achievable HBM rate."""
    import torch
    n = (1 << 31) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / reps * 1e-3
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 4 / s / 1e9


def cpu_baseline(n, fields, steps):
    import oracle
    lat = oracle.Lattice(2, n, n, omega=1.8)
    f = lat.init(*fields)
    t = time.perf_counter()
    f = lat.step(f, steps)
    dt = time.perf_counter() - t
    return {"value": n * n * steps / dt / 1e6, "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps of the same {n}x{n} KH lattice, FP64 C oracle "
                      f"(OpenMP), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on exactly one GPU; the multi-GPU "
              "(y-slab halo exchange) path is design-only, so --gpus N>1 is not "
              "measured.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1402_5487_amd import inputs

    n = args.size
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, delta=n / 80.0, theta=args.theta)
    forms = args.forms.split(",") if args.only is None else [args.only]
    results, moms = {}, {}
    for storage in forms:
        print(f"[bench] timing {storage} {n}x{n} steps={args.steps}", file=sys.stderr,
              flush=True)
        lat, res, mom = time_form(storage, n, fields, args.steps, args.warmup, args.theta)
        results[storage] = res
        moms[storage] = mom
        del lat
        torch.cuda.empty_cache()
    if args.only is not None:
        print(json.dumps({"form": args.only, **results[args.only]}), flush=True)
        return
    # errors of each form against the FP64 form after the same steps
    if "f64" in moms:
        ref = moms["f64"]
        for storage, mom in moms.items():
            results[storage]["max_abs_err_vs_f64_after_steps"] = {
                "steps": args.warmup + args.steps,
                "rho": float((mom[0] - ref[0]).abs().max()),
                "ux": float((mom[1] - ref[1]).abs().max()),
                "uy": float((mom[2] - ref[2]).abs().max()),
                "theta": float((mom[3] - ref[3]).abs().max()),
                "finite": bool(torch.isfinite(mom[0]).all()),
            }
    moms.clear()
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth()

    head = "f16dev" if "f16dev" in results else forms[0]
    h = results[head]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_sha256_16") == kernel_hash() and head in tr.get("forms", {}):
            traffic = tr["forms"][head]["hbm_bytes_per_launch"]
    cpu = None
    if not args.no_cpu:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(n, fields, args.cpu_steps)

    storage_dtype = {"f64": "f64", "f32": "f32", "f16dev": "f32", "bf16dev": "f32"}
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
        "dtype": storage_dtype[head],
        "data": "synthetic",
        "config": {"workload": f"D2Q25 thermal KH {n}x{n} periodic, {head} storage",
                   "nx": n, "ny": n, "storage": head, "theta": args.theta,
                   "omega": 1.8, "u0": 0.1},
        "roofline": {"bound": "hbm", "achieved": round(h["gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(h["frac"], 4), "traffic": traffic},
        "cpu_baseline": cpu,
        "forms": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in results.items()},
        "copy_gbs": round(copy_gbs, 1),
        "copy_frac": round(copy_gbs / HBM_PEAK_GBS, 4),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
