"""Lattice objects over libplbm: torch owns the device buffers and streams.

A Lattice holds one plbm_desc and the two population buffers of the pull
scheme; every operation is one C-ABI call into the HIP library.
"""
import numpy as np
import torch

from . import _plbm

_TORCH_DTYPE = {_plbm.PLBM_F64: torch.float64, _plbm.PLBM_F32: torch.float32,
                _plbm.PLBM_F16DEV: torch.float16, _plbm.PLBM_BF16DEV: torch.bfloat16}


def _dev_f64(a, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


class Lattice:
    """D1Q5 (dim 1, zero-gradient ends) or D2Q25 (dim 2, periodic) lattice of
    the thermal five-velocity model, or (zeta given) the isothermal D1Q3 /
    D2Q9 lattice of the three-velocity family with theta0 = 1 / zeta, or
    (velocities given) the model of any on-lattice set of 3 to 7 velocities
    (isothermal at theta0 for up to four, thermal beyond).

    storage: "f64", "f32", "f16dev" or "bf16dev" (16-bit deviations from the
    rest state rho0 w_k with per-plane power-of-two scales; D2Q25 only).
    rounding: "nearest" or "stochastic" (16-bit deviations only).
    """

    def __init__(self, dim, nx, ny=1, omega=1.0, storage="f64", device="cuda:0",
                 rho0=1.0, theta0=None, zeta=None, velocities=None, rounding="nearest"):
        self.device = torch.device(device)
        if zeta is not None:
            self.desc = _plbm.desc_q3(dim, nx, ny, omega, storage, zeta=zeta)
        elif velocities is not None:
            self.desc = _plbm.desc_general(dim, nx, ny, omega, storage, velocities, theta0)
        else:
            self.desc = _plbm.desc_default(dim, nx, ny, omega, storage)
        if theta0 is not None:
            self.desc.theta0 = float(theta0)
        self.desc.rho0 = float(rho0)
        self.desc.rounding = _plbm.ROUNDING[rounding]
        if _plbm.buffer_elems(self.desc) == 0:
            raise _plbm.PlbmError(_plbm.PLBM_EINVAL, "Lattice: rounding needs 16-bit storage")
        self.dim, self.nx, self.ny = dim, nx, (1 if dim == 1 else ny)
        self.dtype = _TORCH_DTYPE[self.desc.storage]
        n = _plbm.buffer_elems(self.desc)
        self.bufs = [torch.empty(n, dtype=self.dtype, device=self.device),
                     torch.empty(n, dtype=self.dtype, device=self.device)]
        self.cur = 0
        self.t = 0

    # -- helpers ---------------------------------------------------------
    @property
    def stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    @property
    def f(self):
        """The current population buffer (post-collision of the last step)."""
        return self.bufs[self.cur]

    @property
    def bytes_per_step(self):
        """Algorithmic HBM bytes of one step: every population read and
        written once."""
        q = self.desc.q1d ** self.dim
        return 2 * q * self.nx * self.ny * _plbm.elem_bytes(self.desc)

    def _fields(self, rho, ux, uy, theta):
        rho, ux, theta = (_dev_f64(a, self.device) for a in (rho, ux, theta))
        uy = None if (self.dim == 1 or uy is None) else _dev_f64(uy, self.device)
        if self.dim == 2 and uy is None:
            uy = torch.zeros_like(rho)
        return rho, ux, uy, theta

    # -- the C ABI -------------------------------------------------------
    def init(self, rho, ux, uy, theta, choose_scales=True):
        rho, ux, uy, theta = self._fields(rho, ux, uy, theta)
        if self.desc.storage >= _plbm.PLBM_F16DEV and choose_scales:
            _plbm.dev_scales(self.desc, rho, ux, uy, theta, self.stream)
        _plbm.init(self.desc, rho, ux, uy, theta, self.f, self.stream)
        self.t = 0
        return self

    def step(self, nsteps=1, sums=False):
        fa, fb = self.bufs[self.cur], self.bufs[1 - self.cur]
        out = _plbm.step(self.desc, fa, fb, nsteps, sums, self.stream)
        if nsteps % 2 == 1:
            self.cur = 1 - self.cur
        self.t += nsteps
        return out

    def step_fields(self, nsteps=1, out=None):
        """nsteps steps (2D D2Q25), the first also writing (rho, ux, uy, theta)
        of the state it reads, i.e. moments() before the call, at no extra
        read.  out: None or four float64 (ny, nx) device tensors."""
        if out is None:
            out = tuple(torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
                        for _ in range(4))
        fa, fb = self.bufs[self.cur], self.bufs[1 - self.cur]
        _plbm.step_fields(self.desc, fa, fb, nsteps, *out, self.stream)
        if nsteps % 2 == 1:
            self.cur = 1 - self.cur
        self.t += nsteps
        return tuple(out)

    def moments(self, sums=False):
        """(rho, ux, uy, theta) of the current pre-collision state as float64
        device tensors shaped (ny, nx) (1D: (nx,), uy None)."""
        shp = (self.nx,) if self.dim == 1 else (self.ny, self.nx)
        out = [torch.empty(shp, dtype=torch.float64, device=self.device) for _ in range(4)]
        if self.dim == 1:
            out[2] = None
        s = _plbm.moments(self.desc, self.f, out[0], out[1], out[2], out[3], sums,
                          self.stream)
        return (tuple(out), s) if sums else tuple(out)

    def sums(self):
        """FP64 (sum f, sum f vx, sum f vy, sum f |v|^2) of the current state."""
        return _plbm.moments(self.desc, self.f, None, None, None, None, True, self.stream)

    # -- checkpoint ------------------------------------------------------
    def state_dict(self):
        return {"f": self.f.detach().clone(), "t": self.t,
                "scale": list(self.desc.scale), "rho0": self.desc.rho0,
                "theta0": self.desc.theta0}

    def load_state_dict(self, st):
        self.f.copy_(st["f"])
        self.t = st["t"]
        for k, s in enumerate(st["scale"]):
            self.desc.scale[k] = s
        self.desc.rho0, self.desc.theta0 = st["rho0"], st["theta0"]


class Lattice3:
    """D3Q125 lattice (Sec. 2.4: the D1Q5 rule {0, +-1, +-3} along three
    axes), periodic, FP64 or FP32 storage.  Fields are (nz, ny, nx) arrays,
    x fastest."""

    def __init__(self, nx, ny, nz, omega=1.0, storage="f64", device="cuda:0"):
        self.device = torch.device(device)
        self.desc = _plbm.desc_3d(nx, ny, nz, omega, storage)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dtype = _TORCH_DTYPE[self.desc.storage]
        n = _plbm.buffer_elems(self.desc)
        self.bufs = [torch.empty(n, dtype=self.dtype, device=self.device),
                     torch.empty(n, dtype=self.dtype, device=self.device)]
        self.cur = 0
        self.t = 0

    @property
    def stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    @property
    def f(self):
        return self.bufs[self.cur]

    @property
    def bytes_per_step(self):
        return 2 * 125 * self.nx * self.ny * self.nz * _plbm.elem_bytes(self.desc)

    def init(self, rho, ux, uy, uz, theta):
        a = [_dev_f64(x, self.device) for x in (rho, ux, uy, uz, theta)]
        _plbm.init3(self.desc, *a, self.f, self.stream)
        self.t = 0
        return self

    def step(self, nsteps=1, sums=False):
        """nsteps fused steps; with sums, the FP64 (sum f, sum f vx,
        sum f vy, sum f |v|^2, sum f vz) of the state they leave."""
        out = _plbm.step(self.desc, self.bufs[self.cur], self.bufs[1 - self.cur], nsteps, sums,
                         self.stream)
        if nsteps % 2 == 1:
            self.cur = 1 - self.cur
        self.t += nsteps
        return out

    def moments(self):
        """(rho, ux, uy, uz, theta) of the current pre-collision state, float64
        device tensors shaped (nz, ny, nx)."""
        out = [torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
               for _ in range(5)]
        _plbm.moments3(self.desc, self.f, *out, False, self.stream)
        return tuple(out)

    def sums(self):
        return _plbm.moments3(self.desc, self.f, None, None, None, None, None, True, self.stream)

