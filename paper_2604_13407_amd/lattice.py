"""Python binding of liblbm.so (the C-ABI in include/pplbm.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides the device memory (the population arrays, the
workspace, masks and outputs) and the stream; the library receives raw
pointers and the stream handle.  There is no CPU fallback: without the built
library or a GPU, constructing a Lattice raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Optional

import numpy as np
import torch

from . import build as _build

LBM_OK = 0
ERRORS = {-1: "LBM_ERR_INVALID_ARG", -2: "LBM_ERR_HIP", -3: "LBM_ERR_NONFINITE", -4: "LBM_ERR_EOS_DOMAIN",
          -5: "LBM_ERR_UNSUPPORTED", -6: "LBM_ERR_STATE"}
FP64, FP32_DEV = 0, 1
KERNEL_FUSED, KERNEL_TWO_PASS = 0, 1
EOS_VDW, EOS_CS = 0, 1
SCHEME_ORIGINAL, SCHEME_IMPROVED = 0, 1
Q2_DEFAULT, Q2_NEG_Q1, Q2_NEG_HALF_Q1 = 0, 1, 2
FORCE_CONST, FORCE_BUOYANT = 0, 1
LOSS_DRAG, LOSS_UERR = 0, 1

RED_FIELDS = ("mass", "mom_x", "mom_y", "wall_x", "wall_y", "uc_num", "uc_den", "buoy", "pphi", "faults")

# Every symbol include/pplbm.h declares.
EXPORTS = ("lbm_abi_version", "lbm_state_bytes", "lbm_workspace_bytes", "lbm_create", "lbm_destroy",
           "lbm_last_error", "lbm_set_eos", "lbm_set_G", "lbm_set_relaxation", "lbm_set_scheme",
           "lbm_set_body_force", "lbm_set_phase_densities", "lbm_set_walls", "lbm_init_equilibrium", "lbm_step",
           "lbm_set_rows_per_wave", "lbm_set_masked_strips",
           "lbm_step_count", "lbm_read_fields", "lbm_reduce", "lbm_state_ptr", "lbm_get_state", "lbm_set_state",
           "lbm_rereference", "lbm_set_rereference_every", "lbm_adjoint_workspace_bytes", "lbm_adjoint_forward",
           "lbm_adjoint_backward", "lbm_create_static")


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
                ("precision", C.c_int32), ("kernel", C.c_int32), ("rho_ref", C.c_double),
                ("log_capacity", C.c_int32), ("reserved", C.c_int32)]


class Buffers(C.Structure):
    _fields_ = [("f_a", C.c_void_p), ("f_b", C.c_void_p), ("workspace", C.c_void_p), ("mask", C.c_void_p),
                ("wall_u", C.c_void_p)]


class Reduction(C.Structure):
    _fields_ = [(n, C.c_double) for n in RED_FIELDS] + [("step", C.c_int64)]

    def as_dict(self) -> Dict[str, float]:
        d = {n: getattr(self, n) for n in RED_FIELDS}
        d["step"] = int(self.step)
        return d


class AdjointConfig(C.Structure):
    _fields_ = [("n_steps", C.c_int64), ("window", C.c_int64), ("loss", C.c_int32), ("checkpoint_every", C.c_int32),
                ("u_target_dev", C.c_void_p)]


_lib = None


def lib():
    """Loads liblbm.so (building it first only if it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.lbm_abi_version.restype = C.c_int
        L.lbm_state_bytes.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
        L.lbm_workspace_bytes.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
        L.lbm_create.argtypes = [C.POINTER(Config), C.POINTER(Buffers), vp, C.POINTER(vp)]
        L.lbm_create_static.argtypes = [C.POINTER(Config), C.POINTER(Buffers), vp, C.POINTER(vp)]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_set_eos.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
        L.lbm_set_G.argtypes = [vp, C.c_double]
        L.lbm_set_relaxation.argtypes = [vp, dp]
        L.lbm_set_scheme.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32]
        L.lbm_set_body_force.argtypes = [vp, C.c_int32, C.c_double, C.c_double]
        L.lbm_set_phase_densities.argtypes = [vp, C.c_double, C.c_double]
        L.lbm_set_walls.argtypes = [vp, C.c_double]
        L.lbm_init_equilibrium.argtypes = [vp, vp, vp, vp]
        L.lbm_step.argtypes = [vp, C.c_int64, C.c_int32, C.POINTER(Reduction), C.c_int64]
        L.lbm_step_count.argtypes = [vp, C.POINTER(C.c_int64)]
        L.lbm_set_rows_per_wave.argtypes = [vp, C.c_int32]
        L.lbm_set_masked_strips.argtypes = [vp, C.c_int32]
        L.lbm_read_fields.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.lbm_reduce.argtypes = [vp, C.POINTER(Reduction)]
        L.lbm_state_ptr.argtypes = [vp, C.POINTER(vp)]
        L.lbm_get_state.argtypes = [vp, vp]
        L.lbm_set_state.argtypes = [vp, vp, C.c_int64]
        L.lbm_rereference.argtypes = [vp]
        L.lbm_set_rereference_every.argtypes = [vp, C.c_int64]
        L.lbm_adjoint_workspace_bytes.argtypes = [C.POINTER(Config), C.POINTER(AdjointConfig), C.POINTER(C.c_size_t)]
        L.lbm_adjoint_forward.argtypes = [vp, C.POINTER(AdjointConfig), vp, vp, C.c_size_t, dp]
        L.lbm_adjoint_backward.argtypes = [vp, vp, dp, dp]
        _lib = L
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(a, device, dtype) -> Optional[torch.Tensor]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a))
    return a.to(device=device, dtype=dtype).contiguous()


class Lattice:
    """One lattice on one GPU.  All device memory is owned by torch tensors held here."""

    def __init__(self, nx: int, ny: int, periodic_x: bool = True, periodic_y: bool = True,
                 precision: int = FP64, kernel: int = KERNEL_FUSED, rho_ref: float = 0.0, mask=None, wall_u=None,
                 device: str = "cuda:0", log_capacity: int = 4096, stream: Optional[torch.cuda.Stream] = None,
                 static_workspace: bool = False):
        """static_workspace: the handle uses the library's static device workspace
        (lbm_create_static) instead of a workspace tensor allocated here."""
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a GPU: torch.cuda.is_available() is False")
        self.device = torch.device(device)
        self.nx, self.ny = nx, ny
        self.precision = precision
        self.cfg = Config(nx, ny, int(periodic_x), int(periodic_y), precision, kernel, float(rho_ref),
                          int(log_capacity), 0)
        L = lib()
        sb, wb = C.c_size_t(0), C.c_size_t(0)
        self._check(L.lbm_state_bytes(C.byref(self.cfg), C.byref(sb)), None)
        self._check(L.lbm_workspace_bytes(C.byref(self.cfg), C.byref(wb)), None)
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        # rows of planes, [ny][planes][nx]: 9 populations; float storage adds a
        # run of per-node reference offsets
        planes = sb.value // (nx * ny * (8 if precision == FP64 else 4))
        self.f_a = torch.empty((ny, planes, nx), dtype=self.dtype, device=self.device)
        self.f_b = torch.empty((ny, planes, nx), dtype=self.dtype, device=self.device)
        assert self.f_a.numel() * self.f_a.element_size() == sb.value
        # torch's caching allocator returns >= 512-byte aligned blocks
        self.workspace = None if static_workspace else torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self.mask = _dev(mask, self.device, torch.uint8)
        self.wall_u = _dev(wall_u, self.device, torch.float64)
        if self.mask is not None:
            assert tuple(self.mask.shape) == (ny, nx)
        if self.wall_u is not None:
            assert tuple(self.wall_u.shape) == (2, ny, nx)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.buf = Buffers(self.f_a.data_ptr(), self.f_b.data_ptr(),
                           None if self.workspace is None else self.workspace.data_ptr(),
                           None if self.mask is None else self.mask.data_ptr(),
                           None if self.wall_u is None else self.wall_u.data_ptr())
        h = C.c_void_p(0)
        with torch.cuda.device(self.device):
            create = L.lbm_create_static if static_workspace else L.lbm_create
            rc = create(C.byref(self.cfg), C.byref(self.buf), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, L.lbm_last_error(None).decode())
        self.h = h

    # ------------------------------------------------------------ plumbing
    def _check(self, rc: int, h):
        if rc != LBM_OK:
            raise LbmError(rc, lib().lbm_last_error(h).decode())

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.lbm_destroy(h)
            self.h = None

    # ------------------------------------------------------------ parameters
    def set_eos(self, kind: int, a: float, b: float, R: float, T: float, k_eos: float = 1.0):
        self._check(lib().lbm_set_eos(self.h, kind, a, b, R, T, k_eos), self.h)

    def set_G(self, G: float):
        self._check(lib().lbm_set_G(self.h, G), self.h)

    def set_relaxation(self, s):
        arr = (C.c_double * 9)(*[float(v) for v in s])
        self._check(lib().lbm_set_relaxation(self.h, arr), self.h)

    def set_scheme(self, scheme: int, eps: float, k1: Optional[float] = None, k2: Optional[float] = None,
                   q2_policy: int = Q2_DEFAULT):
        k1 = math.nan if k1 is None else k1
        k2 = math.nan if k2 is None else k2
        self._check(lib().lbm_set_scheme(self.h, scheme, eps, k1, k2, q2_policy), self.h)

    def set_body_force(self, mode: int, fx: float, fy: float):
        self._check(lib().lbm_set_body_force(self.h, mode, fx, fy), self.h)
        self.force = (mode, float(fx), float(fy))

    def set_force_magnitude(self, mag: float):
        """Rescales the body force / gravity to magnitude mag, keeping its mode and direction."""
        mode, fx, fy = self.force
        n = math.hypot(fx, fy)
        if n == 0.0:
            raise ValueError("the body force has no direction to rescale")
        self.set_body_force(mode, fx * mag / n, fy * mag / n)

    def set_phase_densities(self, rho_g: float, rho_l: float):
        self._check(lib().lbm_set_phase_densities(self.h, rho_g, rho_l), self.h)

    def set_walls(self, rho_s: float):
        self._check(lib().lbm_set_walls(self.h, rho_s), self.h)

    def set_rows_per_wave(self, rows: int):
        """Launch tuning of the fused kernels (0 = default); results do not depend on it."""
        self._check(lib().lbm_set_rows_per_wave(self.h, rows), self.h)

    def set_masked_strips(self, on: bool):
        """Masked lattices: the masked strip march (True, default; double storage of
        widths that are not a multiple of 64 only on lattices that stream from HBM)
        or the tile kernel (False)."""
        self._check(lib().lbm_set_masked_strips(self.h, 1 if on else 0), self.h)

    # ------------------------------------------------------------ state
    def init_equilibrium(self, rho0, ux0=None, uy0=None):
        r = _dev(rho0, self.device, torch.float64)
        u = _dev(ux0, self.device, torch.float64)
        v = _dev(uy0, self.device, torch.float64)
        assert tuple(r.shape) == (self.ny, self.nx)
        self._keep = (r, u, v)  # alive until the enqueued kernel has read them
        self._check(lib().lbm_init_equilibrium(self.h, _ptr(r), _ptr(u), _ptr(v)), self.h)

    def step(self, n: int, reduce_every: int = 0) -> List[Dict[str, float]]:
        if reduce_every > 0:
            cnt = self.step_count
            nrec = (cnt + n) // reduce_every - cnt // reduce_every
            out = (Reduction * max(nrec, 1))()
            self._check(lib().lbm_step(self.h, n, reduce_every, out, nrec), self.h)
            return [out[i].as_dict() for i in range(nrec)]
        self._check(lib().lbm_step(self.h, n, 0, None, 0), self.h)
        return []

    @property
    def step_count(self) -> int:
        v = C.c_int64(0)
        self._check(lib().lbm_step_count(self.h, C.byref(v)), self.h)
        return v.value

    def rereference(self):
        """Float storage: make every node's reference density its current density."""
        self._check(lib().lbm_rereference(self.h), self.h)

    def set_rereference_every(self, k: int):
        """Float storage: step() re-references after every step whose count is a multiple
        of k (0: never; default 1000)."""
        self._check(lib().lbm_set_rereference_every(self.h, k), self.h)

    def state(self) -> torch.Tensor:
        """The current state as a [planes][ny][nx] view of the array that holds it: 9
        population planes (FP32_DEV: stored relative to the reference densities whose
        offsets, as 16-bit floats, plane 9 holds)."""
        p = C.c_void_p(0)
        self._check(lib().lbm_state_ptr(self.h, C.byref(p)), self.h)
        f = self.f_a if p.value == self.f_a.data_ptr() else self.f_b
        return f.permute(1, 0, 2)

    def get_state(self) -> torch.Tensor:
        """A copy of the state in the library's layout ([ny][planes][nx]), for set_state."""
        dst = torch.empty_like(self.f_a)
        self._check(lib().lbm_get_state(self.h, _ptr(dst)), self.h)
        return dst

    def set_state(self, src: torch.Tensor, step: int = 0):
        src = src.to(device=self.device, dtype=self.dtype).contiguous()
        self._keep = (src,)
        self._check(lib().lbm_set_state(self.h, _ptr(src), step), self.h)

    def read_fields(self) -> Dict[str, torch.Tensor]:
        """Pre-collision fields of the current state: rho, ux, uy, fintx, finty, psi (FP64, device)."""
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "fintx", "finty", "psi")}
        self._check(lib().lbm_read_fields(self.h, _ptr(out["rho"]), _ptr(out["ux"]), _ptr(out["uy"]),
                                          _ptr(out["fintx"]), _ptr(out["finty"]), _ptr(out["psi"])), self.h)
        return out

    def reduce(self) -> Dict[str, float]:
        r = Reduction()
        self._check(lib().lbm_reduce(self.h, C.byref(r)), self.h)
        return r.as_dict()

    # ------------------------------------------------------------ adjoint
    def adjoint_forward(self, rho0, n_steps: int, loss: int = LOSS_DRAG, window: int = 2,
                        checkpoint_every: int = 100, u_target=None) -> float:
        """Runs n_steps from rest with density rho0, saving checkpoints, and returns the loss
        (LOSS_DRAG over the last `window` steps, or LOSS_UERR against u_target).  The lattice
        then holds the state after the run; adjoint_backward() gives the gradients."""
        r = _dev(rho0, self.device, torch.float64)
        assert tuple(r.shape) == (self.ny, self.nx)
        ut = _dev(u_target, self.device, torch.float64)
        if loss == LOSS_UERR:
            assert ut is not None and tuple(ut.shape) == (self.ny, self.nx)
        acfg = AdjointConfig(int(n_steps), int(window), int(loss), int(checkpoint_every),
                             None if ut is None else ut.data_ptr())
        nb = C.c_size_t(0)
        self._check(lib().lbm_adjoint_workspace_bytes(C.byref(self.cfg), C.byref(acfg), C.byref(nb)), None)
        ws = getattr(self, "_adj_ws", None)
        if ws is None or ws.numel() < nb.value:
            self._adj_ws = None
            ws = self._adj_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        assert ws.data_ptr() % 256 == 0
        out = C.c_double(0.0)
        # the library keeps acfg's contents and u_target's pointer for adjoint_backward
        self._adj_keep = (r, ut, acfg)
        self._check(lib().lbm_adjoint_forward(self.h, C.byref(acfg), _ptr(r), _ptr(ws), ws.numel(), C.byref(out)),
                    self.h)
        return out.value

    def adjoint_backward(self):
        """Gradients of the last adjoint_forward's loss: (dL/drho0 [ny, nx] FP64 device tensor,
        dL/d|F_ext|, dL/dG)."""
        g = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        gf, gG = C.c_double(0.0), C.c_double(0.0)
        self._check(lib().lbm_adjoint_backward(self.h, _ptr(g), C.byref(gf), C.byref(gG)), self.h)
        return g, gf.value, gG.value

    # ------------------------------------------------------------ convenience
    @classmethod
    def from_workload(cls, w, precision: int = FP64, kernel: int = KERNEL_FUSED, rho_ref: Optional[float] = None,
                      device: str = "cuda:0", init: bool = True, **kw) -> "Lattice":
        """A lattice with the parameters and seeded inputs of a workloads.Workload."""
        if rho_ref is None:
            rho_ref = w.rho_g if precision == FP32_DEV else 0.0
        lat = cls(w.nx, w.ny, w.periodic_x, w.periodic_y, precision, kernel, rho_ref, mask=w.mask(),
                  wall_u=w.wall_velocity(), device=device, **kw)
        lat.set_eos(w.eos_kind, w.a, w.b, w.R, w.T, w.k_eos)
        lat.set_G(w.G)
        lat.set_relaxation(w.s)
        lat.set_scheme(w.scheme, w.eps, w.k1, w.k2)
        lat.set_body_force(w.force_mode, w.fx, w.fy)
        lat.set_phase_densities(w.rho_g, w.rho_l)
        lat.set_walls(w.rho_s)
        if init:
            lat.init_equilibrium(w.rho0())
        return lat
