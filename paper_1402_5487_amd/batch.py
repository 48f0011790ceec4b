"""Batching form over libplbm: many independent lattices, one launch per step.

The library owns the device pool of all population buffers and the captured
hipGraph; torch supplies the stream and the field tensors handed to init.
"""
import ctypes

import numpy as np
import torch

from . import _plbm


def _dev_f64(a, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


class Batch:
    """`specs`: list of (nx, ny, omega).  FP32 storage, D2Q25, periodic."""

    def __init__(self, specs, device="cuda:0"):
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.proto = _plbm.desc_default(2, 64, 64, 1.5, "f32")
        arr = (_plbm.LatticeSpec * len(specs))(
            *[_plbm.LatticeSpec(int(nx), int(ny), float(om)) for nx, ny, om in specs])
        h = ctypes.c_void_p()
        _plbm.check(_plbm.lib.plbm_batch_create(ctypes.byref(self.proto), arr, len(specs),
                                                ctypes.byref(h)), "plbm_batch_create")
        self.handle = h
        self.specs = [tuple(s) for s in specs]

    def close(self):
        if self.handle:
            _plbm.lib.plbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def autotune(self, cache_path=None):
        p = None if cache_path is None else str(cache_path).encode()
        _plbm.check(_plbm.lib.plbm_batch_autotune(self.handle, p, ctypes.c_void_p(self.stream)),
                    "plbm_batch_autotune")

    def set_graph_steps(self, n):
        _plbm.check(_plbm.lib.plbm_batch_set_graph_steps(self.handle, int(n)),
                    "plbm_batch_set_graph_steps")

    def init(self, i, rho, ux, uy, theta):
        t = [_dev_f64(a, self.device) for a in (rho, ux, uy, theta)]
        _plbm.check(_plbm.lib.plbm_batch_init(self.handle, int(i), *[_plbm._ptr(a) for a in t],
                                              ctypes.c_void_p(self.stream)), "plbm_batch_init")
        self._keep = t            # fields must live until the async init ran
        return self

    def step(self, nsteps):
        _plbm.check(_plbm.lib.plbm_batch_step(self.handle, int(nsteps),
                                              ctypes.c_void_p(self.stream)), "plbm_batch_step")

    def moments(self, i, sums=False):
        nx, ny, _ = self.specs[i]
        out = [torch.empty((ny, nx), dtype=torch.float64, device=self.device) for _ in range(4)]
        s = (ctypes.c_double * 4)() if sums else None
        _plbm.check(_plbm.lib.plbm_batch_moments(self.handle, int(i), *[_plbm._ptr(a) for a in out],
                                                 s, ctypes.c_void_p(self.stream)),
                    "plbm_batch_moments")
        return (tuple(out), list(s)) if sums else tuple(out)

    def buffer(self, i):
        """Current population buffer of lattice i as a float32 tensor view."""
        nx, ny, _ = self.specs[i]
        f = ctypes.c_void_p()
        _plbm.check(_plbm.lib.plbm_batch_lattice(self.handle, int(i), None, ctypes.byref(f)),
                    "plbm_batch_lattice")
        n = 25 * nx * ny
        n4 = (n + 3) // 4 * 4        # buffers are 256-byte aligned with slack
        cpy = torch.empty(n4, dtype=torch.float32, device=self.device)
        _plbm.check(_plbm.lib.plbm_stream_copy(f, _plbm._ptr(cpy), n4 * 4,
                                               ctypes.c_void_p(self.stream)), "copy")
        return cpy[:n]

    def info(self):
        inf = _plbm.BatchInfo()
        _plbm.check(_plbm.lib.plbm_batch_query(self.handle, ctypes.byref(inf)), "plbm_batch_query")
        classes = {inf.class_size[k]: (inf.class_w[k], inf.class_r[k]) for k in range(inf.classes)}
        return {"count": inf.count, "tiles": inf.tiles, "grid_mode": inf.grid_mode,
                "lds_bytes": inf.lds_bytes, "graph_steps": inf.graph_steps,
                "parity": inf.parity, "nodes": inf.nodes, "pool_bytes": inf.pool_bytes,
                "classes": classes}
