"""The benchmark's command-line contract, checked without a GPU: more than
one GPU is refused with a message, the CPU baseline leg reports what the
result line needs, and every default form names its arithmetic type."""
import os
import json
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1402_5487_amd import inputs  # noqa: E402


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, env=e)


def test_more_than_one_gpu_is_refused():
    for args, env in ((["--gpus", "2"], None), (["--gpus", "8"], None), ([], {"WORLD_SIZE": "2"})):
        r = _run(args, env)
        assert r.returncode != 0
        assert "one GPU" in r.stderr
        assert r.stdout.strip() == ""          # no result line


def test_cpu_baseline_leg():
    n = 24
    fields = inputs.kelvin_helmholtz(n, n, u0=0.1, theta=0.35)
    out, ref = bench.cpu_baseline(n, fields, 2)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS"
    assert out["value"] > 0 and np.isfinite(out["value"])
    assert out["one_thread_mlups"] > 0
    assert isinstance(out["cores"], int) and out["cores"] >= 1
    assert "steps" in out["sample"]
    # the moments handed to the FP64 anchor are the oracle's after the steps
    import oracle
    lat = oracle.Lattice(2, n, n, omega=1.8)
    want = lat.moments(lat.step(lat.init(*fields), 2))
    assert all(np.array_equal(a, b) for a, b in zip(ref, want))
    assert oracle.num_threads() == out["cores"]     # thread count restored


def test_default_forms_have_a_compute_dtype(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    args = bench.parse()
    for f in args.forms.split(","):
        assert f in bench.COMPUTE_DTYPE
    assert args.gpus == 1 and args.steps > 0 and args.warmup >= 0


def test_kernel_hash_is_stable():
    assert bench.kernel_hash() == bench.kernel_hash()
    assert len(bench.kernel_hash()) == 16


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path):
    good = {"kernel_sha256_16": bench.kernel_hash(),
            "forms": {"f16dev": {"hbm_bytes_per_launch": 123}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    assert bench.stored_traffic("f16dev", str(p)) == 123
    assert bench.stored_traffic("f32", str(p)) is None
    p.write_text(json.dumps(dict(good, kernel_sha256_16="0" * 16)))
    assert bench.stored_traffic("f16dev", str(p)) is None
    assert bench.stored_traffic("f16dev", str(tmp_path / "missing.json")) is None


def test_stored_counters_match_the_algorithmic_bytes():
    """The committed counter totals: every step form moves its algorithmic
    bytes (50 populations of its element size per node, 4096^2 nodes) to
    within 3 %."""
    with open(bench.TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    for form, v in tr["forms"].items():
        assert v["algorithmic_bytes_per_launch"] == 50 * {"f64": 8, "f32": 4}.get(form, 2) * 4096 ** 2
        assert abs(v["hbm_over_algorithmic"] - 1) < 0.03, form


def test_first_nonfinite_stops_at_the_reported_step():
    from paper_1402_5487_amd import _plbm
    calls = []

    def step(k):
        calls.append(k)
        if sum(calls) >= 75:
            raise _plbm.PlbmError(_plbm.PLBM_ENONFINITE, "plbm_step")
    assert bench.first_nonfinite(step, 1000, 25) == 75
    calls.clear()
    assert bench.first_nonfinite(lambda k: calls.append(k), 100, 25) is None and sum(calls) == 100


def test_literal_predictions_from_the_oracle_growth():
    """The CPU leg's predictions: the literal KH state grows (the oracle's
    von Neumann factor exceeds 1) and each form's predicted blow-up step
    follows its store rounding; a stable batch member (theta = 0.35) is
    predicted never to blow up, an unstable one (theta = 0.25) within the run."""
    lit = {"f64": {"first_nonfinite_step": 550}, "f16dev": {"first_nonfinite_step": 200}}
    bench.predict_literal_kh(lit)
    assert 1.05 < lit["growth_per_step"] < 1.2
    assert lit["f64"]["predicted_step"] > lit["f16dev"]["predicted_step"] > 0
    lb = {"steps": 2000, "_members": [(0.35, 0.05, 1.7), (0.25, 0.1, 1.85)], "_first": [None, 150]}
    bench.predict_literal_batch(lb)
    assert lb["predicted_unstable"] == 1 and lb["agree_with_prediction"] == 2
    assert "_members" not in lb
