"""Learned closure over libplbm: argument marshalling for plbm_closure_* and
plbm_restrict.  Parameters, gradients and Adam moments are torch float32
device tensors of PLBM_CNN_PARAMS entries (layout in include/plbm.h)."""
import ctypes

import torch

from . import _plbm

CNN_PARAMS = _plbm.CNN_PARAMS
LAYER = _plbm.CNN_LAYER_PARAMS
CH = 32


def _ptrs(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def init_params(seed=0, device="cuda:0", out_gain=0.1):
    """He-uniform weights on the real channels (25 inputs of layer 1, 25
    outputs of layer 3), zero in the padding and in the biases."""
    g = torch.Generator().manual_seed(seed)
    p = torch.zeros(CNN_PARAMS, dtype=torch.float32)
    for layer, (cin, cout) in enumerate(((25, 32), (32, 32), (32, 25))):
        w = torch.zeros(9, CH, CH)
        bound = (6.0 / (9 * cin)) ** 0.5 * (out_gain if layer == 2 else 1.0)
        w[:, :cout, :cin] = (torch.rand(9, cout, cin, generator=g) * 2 - 1) * bound
        p[layer * LAYER:layer * LAYER + 9 * CH * CH] = w.reshape(-1)
    return p.to(device)


def split_params(p):
    """Flat vector -> [(w[3,3,in,out], b[out]) x 3] float64 numpy (oracle form)."""
    import numpy as np
    q = p.detach().double().cpu().numpy()
    out = []
    for layer, (cin, cout) in enumerate(((25, 32), (32, 32), (32, 25))):
        w = q[layer * LAYER:layer * LAYER + 9 * CH * CH].reshape(9, CH, CH)   # [t][o][i]
        b = q[layer * LAYER + 9 * CH * CH:(layer + 1) * LAYER]
        wt = np.transpose(w, (0, 2, 1)).reshape(3, 3, CH, CH)                 # [dy][dx][i][o]
        out.append((wt[:, :, :cin, :cout].copy(), b[:cout].copy()))
    return out


class Closure:
    """Network workspaces for up to `frames` coarse nx x ny lattices whose
    populations are stored as `storage` ("f32" or "f64")."""

    def __init__(self, nx, ny, frames, device="cuda:0", storage="f64"):
        self.device = torch.device(device)
        self.desc = _plbm.desc_default(2, nx, ny, 1.9, storage)
        h = ctypes.c_void_p()
        _plbm.check(_plbm.lib.plbm_closure_create(ctypes.byref(self.desc), int(frames),
                                                  ctypes.byref(h)), "plbm_closure_create")
        self.handle = h
        self.nx, self.ny, self.frames = nx, ny, frames
        self._nf = 0

    def close(self):
        if self.handle:
            _plbm.lib.plbm_closure_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_norm(self, in_mean, in_scale, out_scale, moment_scale):
        arr = [(ctypes.c_float * len(a))(*[float(v) for v in a])
               for a in (in_mean, in_scale, out_scale, moment_scale)]
        if [len(a) for a in arr] != [25, 25, 25, 4]:
            raise ValueError("set_norm: 25, 25, 25 and 4 values expected")
        _plbm.check(_plbm.lib.plbm_closure_set_norm(self.handle, *arr), "plbm_closure_set_norm")

    def forward(self, params, posts, noise=None, noise_amp=0.0):
        """noise: None, or a float32 device tensor of frames * 25 * ny * nx
        values (planes [frame][k][y][x]) added, times noise_amp, to the
        normalised input."""
        self._nf = len(posts)
        if noise is not None and (noise.dtype != torch.float32 or
                                  noise.numel() < len(posts) * self.ny * self.nx * 25):
            raise ValueError("forward: float32 noise of frames * ny * nx * 25 values expected")
        _plbm.check(_plbm.lib.plbm_closure_forward(
            self.handle, ctypes.c_void_p(params.data_ptr()), _ptrs(posts), len(posts),
            None if noise is None else ctypes.c_void_p(noise.data_ptr()), float(noise_amp),
            _stream(self.device)), "plbm_closure_forward")

    def backward(self, params, targets, grads, want_loss=True, reg=0.0):
        """targets: per frame, the increment error d as a float32 (4, ny, nx)
        device tensor (see target()); reg: minimum-norm weight."""
        loss = ctypes.c_double() if want_loss else None
        _plbm.check(_plbm.lib.plbm_closure_backward(
            self.handle, ctypes.c_void_p(params.data_ptr()), _ptrs(targets), float(reg),
            ctypes.c_void_p(grads.data_ptr()), ctypes.byref(loss) if want_loss else None,
            _stream(self.device)), "plbm_closure_backward")
        return loss.value if want_loss else None

    def adam(self, params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        _plbm.check(_plbm.lib.plbm_closure_adam(
            self.handle, *[ctypes.c_void_p(a.data_ptr()) for a in (params, grads, m, v)], int(t),
            float(lr), float(b1), float(b2), float(eps), _stream(self.device)), "plbm_closure_adam")

    def apply(self, posts, bound=8.0, skipped=None):
        _plbm.check(_plbm.lib.plbm_closure_apply(
            self.handle, _ptrs(posts), len(posts), float(bound),
            None if skipped is None else ctypes.c_void_p(skipped.data_ptr()),
            _stream(self.device)), "plbm_closure_apply")

    # -- training through coarse steps (adjoints) ---------------------------
    def rollout_loss(self, posts, truths, scale, lams=None, want_loss=True):
        """L = scale sum w_j (m_j - cons_j(truth))^2 over the states `posts`;
        truths: per frame a (rho, ux, uy, theta) tuple of FP64 device fields;
        lams: None or per-frame FP64 adjoint buffers receiving dL/dpost."""
        flat = [t for tr in truths for t in tr]
        loss = ctypes.c_double() if want_loss else None
        _plbm.check(_plbm.lib.plbm_closure_rollout_loss(
            self.handle, _ptrs(posts), _ptrs(flat), len(posts), float(scale),
            None if lams is None else _ptrs(lams), ctypes.byref(loss) if want_loss else None,
            _stream(self.device)), "plbm_closure_rollout_loss")
        return loss.value if want_loss else None

    def apply_vjp(self, posts, lams):
        """Adjoint of apply for the buffers of the last forward (pre-apply);
        lams (dL/dpost') are updated in place through the state path."""
        _plbm.check(_plbm.lib.plbm_closure_apply_vjp(self.handle, _ptrs(posts), _ptrs(lams), len(posts),
                                                     _stream(self.device)), "plbm_closure_apply_vjp")

    def backward_vjp(self, params, grads, accumulate=True, lams=None, reg=0.0):
        """The network's part of the apply adjoint: parameter gradients into
        grads (added when accumulate) and, with lams, the input gradient."""
        _plbm.check(_plbm.lib.plbm_closure_backward_vjp(
            self.handle, ctypes.c_void_p(params.data_ptr()), float(reg), ctypes.c_void_p(grads.data_ptr()),
            1 if accumulate else 0, None if lams is None else _ptrs(lams), _stream(self.device)),
            "plbm_closure_backward_vjp")

    def rollout_vjp(self, desc, params, grads, accumulate, after, truths, scale, pre,
                    before=None, lam_in=None, lam_out=None, want_loss=False, reg=0.0):
        """One fused backward step of rollout training (plbm_closure_rollout_vjp):
        desc the coarse lattice's descriptor; after the states the loss reads,
        truths their (rho, ux, uy, theta) tuples; pre the buffers of the last
        forward; before the buffers the coarse step read; lam_in dL/dafter
        from later steps (None: zero); lam_out receives dL/dbefore (None:
        skipped).  Returns the segment loss so far when want_loss."""
        n = len(after)
        flat = [t for tr in truths for t in tr]
        loss = ctypes.c_double() if want_loss else None
        _plbm.check(_plbm.lib.plbm_closure_rollout_vjp(
            self.handle, ctypes.byref(desc), ctypes.c_void_p(params.data_ptr()), float(reg),
            ctypes.c_void_p(grads.data_ptr()), 1 if accumulate else 0, _ptrs(after), _ptrs(flat),
            float(scale), _ptrs(pre), None if before is None else _ptrs(before),
            None if lam_in is None else _ptrs(lam_in), None if lam_out is None else _ptrs(lam_out),
            n, ctypes.byref(loss) if want_loss else None, _stream(self.device)),
            "plbm_closure_rollout_vjp")
        return loss.value if want_loss else None

    def activation(self, which):
        """Copy of an internal buffer: bf16 NHWC (which 0..2, 4..6) as float32
        (frames, ny, nx, 32), the FP32 output (3), the physical correction
        (7: frames, 25, ny, nx), dL/dm (8: frames, 4, ny, nx), the moment
        cotangents of the last adjoint call (10: frames, 4, ny, nx) or the
        gradient of the network input (11: frames, ny, nx, 32)."""
        ptr, nbytes = ctypes.c_void_p(), ctypes.c_size_t()
        _plbm.check(_plbm.lib.plbm_closure_activation(self.handle, int(which), ctypes.byref(ptr),
                                                      ctypes.byref(nbytes)), "activation")
        nodes = self.frames * self.ny * self.nx
        if which == 10:
            out = torch.empty(nbytes.value // 8, dtype=torch.float64, device=self.device)
        elif which in (3, 7, 8, 11):
            out = torch.empty(nbytes.value // 4, dtype=torch.float32, device=self.device)
        else:
            out = torch.empty(nodes * CH, dtype=torch.bfloat16, device=self.device)
        _plbm.check(_plbm.lib.plbm_stream_copy(ptr, ctypes.c_void_p(out.data_ptr()), nbytes.value,
                                               _stream(self.device)), "copy")
        nf = max(self._nf, 1)
        if which == 7:
            return out.reshape(self.frames, 25, self.ny, self.nx)[:nf]
        if which in (8, 10):
            return out.reshape(self.frames, self.ny, self.nx, 4).permute(0, 3, 1, 2)[:nf]
        if which == 11:
            return out.reshape(self.frames, self.ny, self.nx, CH)[:nf]
        return out.float().reshape(self.frames, self.ny, self.nx, CH)[:nf]


def restrict(rho, ux, uy, theta, factor=4):
    """Coarse (rho, u, theta) from fine FP64 device fields (plbm_restrict)."""
    fny, fnx = rho.shape
    out = [torch.empty((fny // factor, fnx // factor), dtype=torch.float64, device=rho.device)
           for _ in range(4)]
    _plbm.check(_plbm.lib.plbm_restrict(*[ctypes.c_void_p(t.data_ptr()) for t in (rho, ux, uy, theta)],
                                        fnx, fny, factor,
                                        *[ctypes.c_void_p(t.data_ptr()) for t in out],
                                        _stream(rho.device)), "plbm_restrict")
    return tuple(out)


def target(truth_prev, truth_now, model_prev, model_now):
    """Increment error d (float32 (4, ny, nx) device tensor) of one frame from
    four (rho, ux, uy, theta) tuples of FP64 device fields
    (plbm_closure_target)."""
    fields = [t for group in (truth_prev, truth_now, model_prev, model_now) for t in group]
    if len(fields) != 16:
        raise ValueError("target: four (rho, ux, uy, theta) tuples expected")
    shape = fields[0].shape
    for t in fields:
        if t.dtype != torch.float64 or t.shape != shape or not t.is_contiguous():
            raise ValueError("target: contiguous float64 fields of one shape expected")
    out = torch.empty((4,) + tuple(shape), dtype=torch.float32, device=fields[0].device)
    _plbm.check(_plbm.lib.plbm_closure_target(_ptrs(fields), fields[0].numel(),
                                              ctypes.c_void_p(out.data_ptr()),
                                              _stream(fields[0].device)), "plbm_closure_target")
    return out
