"""GPU tests of the batching form (plbm_batch_*): every lattice of a batch
must evolve exactly as the same lattice stepped alone (same FP32 arithmetic,
so bitwise), whatever the tile shapes, grid mode and graph replay, and a
batch lattice must match the FP64 oracle to the FP32 bound."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_1402_5487_amd import inputs
from paper_1402_5487_amd.batch import Batch
from paper_1402_5487_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

SPECS = [(64, 64, 1.6), (96, 96, 1.7), (100, 70, 1.5), (130, 130, 1.85),
         (256, 200, 1.8), (7, 5, 1.3), (300, 41, 1.75)]


def _fields(i, nx, ny):
    return inputs.kelvin_helmholtz(nx, ny, u0=0.03 + 0.01 * i, theta=0.35)


def _single(nx, ny, om, fields, steps):
    lat = Lattice(2, nx, ny, omega=om, storage="f32").init(*fields)
    lat.step(steps)
    return lat.f.clone()


def _run_batch(steps_plan, graph_steps=8, tune=None):
    b = Batch(SPECS)
    if tune is not None:
        b.autotune(tune)
    b.set_graph_steps(graph_steps)
    for i, (nx, ny, _) in enumerate(SPECS):
        b.init(i, *_fields(i, nx, ny))
    for n in steps_plan:
        b.step(n)
    torch.cuda.synchronize()
    return b


@pytest.fixture(scope="module")
def reference():
    return [_single(nx, ny, om, _fields(i, nx, ny), 21) for i, (nx, ny, om) in enumerate(SPECS)]


@pytest.mark.parametrize("graph_steps,plan", [(0, [21]), (8, [21]), (4, [3, 18]), (2, [1, 1, 19])])
def test_batch_equals_single_lattices_bitwise(reference, graph_steps, plan):
    b = _run_batch(plan, graph_steps)
    for i in range(len(SPECS)):
        assert torch.equal(b.buffer(i), reference[i]), i
    b.close()


def test_autotuned_batch_is_bitwise_equal_and_cached(reference, tmp_path):
    cache = tmp_path / "tune.json"
    b = _run_batch([21], 8, tune=cache)
    info = b.info()
    for i in range(len(SPECS)):
        assert torch.equal(b.buffer(i), reference[i]), i
    data = json.loads(cache.read_text())
    classes = {e["class"] for e in data["entries"]}
    assert classes == {max(nx, ny) for nx, ny, _ in SPECS}
    assert set(info["classes"]) == classes
    for w, r in info["classes"].values():
        assert w in (64, 128, 256) and r in (1, 2, 4, 8)
    b.close()
    # a second batch reuses the cached choices
    b2 = _run_batch([21], 8, tune=cache)
    assert b2.info()["classes"] == info["classes"]
    for i in range(len(SPECS)):
        assert torch.equal(b2.buffer(i), reference[i]), i
    b2.close()


def _bitwise_against_single(specs, steps, tune=None, graph_steps=8):
    b = Batch(specs)
    if tune is not None:
        b.autotune(tune)
    b.set_graph_steps(graph_steps)
    for i, (nx, ny, _) in enumerate(specs):
        b.init(i, *_fields(i % 9, nx, ny))
    b.step(steps)
    torch.cuda.synchronize()
    for i, (nx, ny, om) in enumerate(specs):
        ref = _single(nx, ny, om, _fields(i % 9, nx, ny), steps)
        assert torch.equal(b.buffer(i), ref), (i, nx, ny)
    info = b.info()
    b.close()
    return info


@pytest.mark.parametrize("tuned", [False, True])
def test_repeated_sizes_keep_their_own_buffers_and_omega(tuned, tmp_path):
    """Lattices of one size share a shape group (back to back in the pool,
    decoded arithmetically); interleaved in the spec list, each still evolves
    exactly as alone with its own relaxation constant."""
    specs = [(64, 64, 1.6), (96, 96, 1.7), (64, 64, 1.5), (96, 96, 1.85), (64, 64, 1.9),
             (7, 5, 1.3), (96, 96, 1.55), (300, 41, 1.75), (7, 5, 1.45)]
    _bitwise_against_single(specs, 13, tune=(tmp_path / "t.json") if tuned else None)


def test_more_sizes_than_groups_use_the_work_list():
    """More distinct sizes than the group table holds (48): the work-list
    kernel runs, with the same results."""
    specs = [(8 + i, 6 + (i % 3), 1.5 + 0.008 * i) for i in range(50)]
    info = _bitwise_against_single(specs, 11)
    assert info["tiles"] > 0


def test_batch_lattice_matches_oracle():
    steps = 30
    b = _run_batch([steps], 8)
    i = 2
    nx, ny, om = SPECS[i]
    got = [t.cpu().numpy() for t in b.moments(i)]
    ref_lat = oracle.Lattice(2, nx, ny, omega=om)
    ref = ref_lat.moments(ref_lat.step(ref_lat.init(*_fields(i, nx, ny)), steps))
    eps = np.finfo(np.float32).eps
    for a, r, floor in zip(got, ref, (1.0, 0.05, 0.05, 1.0)):
        assert np.abs(a - r).max() / max(np.abs(r).max(), floor) < steps * 200 * eps
    b.close()


def test_batch_conserves_mass_per_lattice():
    b = _run_batch([0], 8)
    s0 = [b.moments(i, sums=True)[1] for i in range(len(SPECS))]
    b.step(40)
    for i in range(len(SPECS)):
        s1 = b.moments(i, sums=True)[1]
        # FP32 storage: rounding of every stored population, not a drift of
        # the method; bounded by steps * eps32 relative
        assert abs(s1[0] / s0[i][0] - 1) < 40 * 2 * np.finfo(np.float32).eps
    b.close()


def _forced_cache(path, specs, mode, w, r, lds=40 * 1024):
    """An autotune cache that fixes every size class's tile shape and the grid
    mode, so the batch runs them without timing anything."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    entries = [{"arch": arch, "storage": "f32", "class": c, "w": w, "r": r}
               for c in sorted({max(nx, ny) for nx, ny, _ in specs})]
    path.write_text(json.dumps({"entries": entries,
                                "grid": {"arch": arch, "mode": mode, "lds": lds}}))
    return path


@pytest.mark.parametrize("mode", [2, 4])
@pytest.mark.parametrize("w,r", [(64, 2), (256, 1)])
def test_persistent_grid_modes_are_bitwise_equal(mode, w, r, tmp_path):
    """Persistent grids (mode k: k workgroups per CU walking the tile list)
    with more tiles than workgroups, so each workgroup runs the tile loop
    several times: still bitwise equal to single lattices."""
    specs = SPECS + [(1024, 1024, 1.75), (512, 512, 1.8), (320, 288, 1.65), (480, 96, 1.7)]
    cache = _forced_cache(tmp_path / "t.json", specs, mode, w, r)
    info = _bitwise_against_single(specs, 9, tune=cache)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert info["grid_mode"] == mode
    assert info["tiles"] > 2 * mode * cus, info["tiles"]
    assert all(v == (w, r) for v in info["classes"].values())


@pytest.mark.parametrize("mode", [2, 4])
def test_persistent_grid_on_the_work_list(mode, tmp_path):
    """More sizes than the group table holds (48) take the device work list;
    with a persistent grid each workgroup walks several work-list tiles."""
    specs = [(100 + 2 * i, 90 + (i % 7), 1.5 + 0.008 * i) for i in range(50)]
    cache = _forced_cache(tmp_path / "t.json", specs, mode, 64, 1)
    info = _bitwise_against_single(specs, 7, tune=cache)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert info["grid_mode"] == mode and info["tiles"] > 2 * mode * cus, info
