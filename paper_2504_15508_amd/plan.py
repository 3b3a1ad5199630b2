"""Python binding of the long-range step: a Plan owning a libdplr_lr plan.

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  PyTorch provides device memory and the current HIP
stream."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib

_DT = {"fp32": torch.float32, "fp64": torch.float64}


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


class Plan:
    """A configured PPPM plan (mesh, order, beta, precision, capacity).

    diff selects the force scheme: "ik" (the paper's Poisson-IK, three
    inverse FFTs) or "ad" (analytic differentiation of the assignment
    weights, one inverse FFT; forces are the exact gradient of the energy).
    compute() returns (energy [0-d float64], ion_force [n_ion,3], wc_force
    [n_wc,3], virial [6] float64) as device tensors; forces are -dE/dr."""

    def __init__(self, mesh, order: int = 5, beta: float = 0.4, coulomb_k: float = 14.399645,
                 precision: str = "fp32", alias_range: int = 2, capacity: int = 0, flags: int = 0,
                 device: Optional[torch.device] = None, diff: str = "ik"):
        lib = _lib.load()
        if diff not in ("ik", "ad"):
            raise ValueError("diff must be 'ik' or 'ad'")
        if diff == "ad":
            flags = int(flags) | _lib.DIFF_AD
        self.diff = diff
        if isinstance(mesh, int):
            mesh = (mesh, mesh, mesh)
        if precision not in _DT:
            raise ValueError("precision must be 'fp32' or 'fp64'")
        self.precision = precision
        self.dtype = _DT[precision]
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        cfg = _lib.Config()
        cfg.mesh[:] = [int(m) for m in mesh]
        cfg.order, cfg.beta, cfg.coulomb_k = int(order), float(beta), float(coulomb_k)
        cfg.precision = _lib.FP64 if precision == "fp64" else _lib.FP32
        cfg.alias_range, cfg.capacity, cfg.flags = int(alias_range), int(capacity), int(flags)
        self.cfg = cfg
        self.mesh, self.order, self.beta, self.coulomb_k = tuple(mesh), int(order), float(beta), float(coulomb_k)
        self.capacity, self.flags = int(capacity), int(flags)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _lib.check(lib.dplr_lr_plan_create(ctypes.byref(cfg), ctypes.c_void_p(stream), ctypes.byref(handle)))
        self._h = handle
        self.box = None
        self.last_virial = None

    def set_fft_int32(self, nodes=None, scale: float = 1e7):
        """The paper's Mixed-Int32 transforms on a mixed-radix plan: node-block
        partial DFTs quantised to int32 at `scale` (see include/dplr_lr.h);
        nodes=None switches them off."""
        lib = _lib.load()
        if nodes is None:
            self._check(lib.dplr_lr_set_fft_int32(self._h, None, 0.0))
            return
        arr = (ctypes.c_int32 * 3)(*[int(v) for v in nodes])
        self._check(lib.dplr_lr_set_fft_int32(self._h, arr, float(scale)))

    # -- plumbing ---------------------------------------------------------
    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.load().dplr_lr_set_stream(self._h, ctypes.c_void_p(s)), self._h)

    def _check(self, st):
        _lib.check(st, self._h)

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.load().dplr_lr_workspace_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().dplr_lr_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API ---------------------------------------------------------------
    def set_box(self, box: Sequence[float]):
        arr = (ctypes.c_double * 3)(*[float(b) for b in box])
        with torch.cuda.device(self.device):
            self._bind_stream()
            self._check(_lib.load().dplr_lr_set_box(self._h, arr))
        self.box = tuple(float(b) for b in box)

    def _as_input(self, t, cols):
        if t is None:
            return torch.empty((0, cols) if cols else (0,), dtype=self.dtype, device=self.device)
        if t.device != self.device or t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError(f"inputs must be contiguous {self.dtype} tensors on {self.device}")
        return t

    def compute(self, ion_pos, ion_q, wc_pos=None, wc_q=None, ion_force=None, wc_force=None,
                energy=None, virial=None):
        ion_pos, ion_q = self._as_input(ion_pos, 3), self._as_input(ion_q, 0)
        wc_pos, wc_q = self._as_input(wc_pos, 3), self._as_input(wc_q, 0)
        n_ion, n_wc = ion_pos.shape[0], wc_pos.shape[0]
        if ion_q.shape[0] != n_ion or wc_q.shape[0] != n_wc:
            raise ValueError("charge and position counts differ")
        dev = self.device
        if ion_force is None:
            ion_force = torch.empty((n_ion, 3), dtype=self.dtype, device=dev)
        if wc_force is None:
            wc_force = torch.empty((n_wc, 3), dtype=self.dtype, device=dev)
        if energy is None:
            energy = torch.empty((), dtype=torch.float64, device=dev)
        if virial is None:
            virial = torch.empty(6, dtype=torch.float64, device=dev)
        with torch.cuda.device(dev):
            self._bind_stream()
            self._check(_lib.load().dplr_lr_compute_energy_forces_virial(
                self._h, n_ion, _ptr(ion_pos), _ptr(ion_q), n_wc, _ptr(wc_pos), _ptr(wc_q),
                _ptr(ion_force), _ptr(wc_force), ctypes.c_void_p(energy.data_ptr()),
                ctypes.c_void_p(virial.data_ptr())))
        return energy, ion_force, wc_force, virial

    def scale_grad(self, grad_energy, ion_force, wc_force, ion_grad=None, wc_grad=None):
        if grad_energy.dtype != torch.float64 or grad_energy.device != self.device:
            grad_energy = grad_energy.to(device=self.device, dtype=torch.float64)
        grad_energy = grad_energy.contiguous()
        if ion_grad is None:
            ion_grad = torch.empty_like(ion_force)
        if wc_grad is None:
            wc_grad = torch.empty_like(wc_force)
        with torch.cuda.device(self.device):
            self._bind_stream()
            self._check(_lib.load().dplr_lr_scale_grad(
                self._h, ctypes.c_void_p(grad_energy.data_ptr()), ion_force.shape[0], _ptr(ion_force),
                _ptr(ion_grad), wc_force.shape[0], _ptr(wc_force), _ptr(wc_grad)))
        return ion_grad, wc_grad

    def profile(self, enable: bool = True):
        """Record HIP events around each kernel of compute (instrumentation)."""
        self._check(_lib.load().dplr_lr_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, reset: bool = True) -> dict:
        """{stage name: (total ms, launches)} since the last reset (synchronises)."""
        import numpy as np
        lib = _lib.load()
        ms = np.zeros(32)
        calls = np.zeros(32, dtype=np.int64)
        n = ctypes.c_int32()
        self._check(lib.dplr_lr_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                             calls.ctypes.data_as(ctypes.c_void_p), 32, ctypes.byref(n),
                                             1 if reset else 0))
        return {lib.dplr_lr_profile_stage_name(i).decode(): (float(ms[i]), int(calls[i]))
                for i in range(n.value)}

    def q32_clamped(self) -> int:
        """Partial values the int32 transforms of the last compute clamped
        (synchronises)."""
        c = self.debug_buffer(_lib.BUF_Q32_CLAMPED)
        torch.cuda.synchronize(self.device)
        return int(c.item())

    def debug_dft_q32(self, axis: int, sign: int, data: torch.Tensor) -> torch.Tensor:
        """One axis of the int32-quantised transform, in place on a complex
        tensor [ncomp][Kz][Ky][Kx] (or [Kz][Ky][Kx]) of the plan's precision."""
        cdt = torch.complex128 if self.precision == "fp64" else torch.complex64
        if data.dtype != cdt or data.device != self.device or not data.is_contiguous():
            raise ValueError(f"data must be a contiguous {cdt} tensor on {self.device}")
        kx, ky, kz = self.mesh
        ncomp = data.numel() // (kx * ky * kz)
        if ncomp * kx * ky * kz != data.numel():
            raise ValueError("data must hold whole [Kz][Ky][Kx] meshes")
        with torch.cuda.device(self.device):
            self._bind_stream()
            self._check(_lib.load().dplr_lr_debug_dft_q32(self._h, int(axis), int(sign),
                                                          ctypes.c_void_p(data.data_ptr()), int(ncomp)))
        return data

    def debug_buffer(self, which: int) -> torch.Tensor:
        """Copy of an intermediate buffer of the last compute (see include/dplr_lr.h)."""
        lib = _lib.load()
        nbytes = int(lib.dplr_lr_debug_size(self._h, which))
        if nbytes < 0:
            raise ValueError(f"buffer {which} is not available on this plan "
                             "(mixed-radix plans keep only the influence table)")
        out = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self._bind_stream()
            self._check(lib.dplr_lr_debug_copy(self._h, which, ctypes.c_void_p(out.data_ptr()), nbytes))
        kx, ky, kz = self.mesh
        kh = kx // 2 + 1
        if which == _lib.BUF_Q32_CLAMPED:
            return out.view(torch.int64)
        if which == _lib.BUF_INFLUENCE:
            return out.view(torch.float64).view(kh, ky // 2 + 1, kz // 2 + 1)
        cdt = torch.complex128 if self.precision == "fp64" else torch.complex64
        c = out.view(cdt)
        if which == _lib.BUF_SPECTRUM:
            return c.view(kh, kz, ky)
        return c.view(3, kh, kz, ky)


def compute_noalloc(mesh, box, ion_pos, ion_q, wc_pos=None, wc_q=None, order: int = 5, beta: float = 0.4,
                    coulomb_k: float = 14.399645, alias_range: int = 2, flags: int = 0, diff: str = "ik",
                    ion_force=None, wc_force=None, energy=None, virial=None):
    """The step through dplr_lr_compute_noalloc: no plan, and no device
    allocation inside the library (its working memory is a fixed device
    array of NOALLOC_SCRATCH_BYTES per GPU).  Precision follows the dtype of
    ion_pos (float32 or float64).  Output tensors that are not given are
    allocated here by PyTorch.  Returns (energy, ion_force, wc_force, virial)."""
    lib = _lib.load()
    dt = ion_pos.dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("positions must be float32 or float64")
    dev = ion_pos.device
    if diff not in ("ik", "ad"):
        raise ValueError("diff must be 'ik' or 'ad'")
    if diff == "ad":
        flags = int(flags) | _lib.DIFF_AD
    if isinstance(mesh, int):
        mesh = (mesh, mesh, mesh)

    def inp(t, cols):
        if t is None:
            return torch.empty((0, cols) if cols else (0,), dtype=dt, device=dev)
        if t.device != dev or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"inputs must be contiguous {dt} tensors on {dev}")
        return t

    ion_pos, ion_q, wc_pos, wc_q = inp(ion_pos, 3), inp(ion_q, 0), inp(wc_pos, 3), inp(wc_q, 0)
    n_ion, n_wc = ion_pos.shape[0], wc_pos.shape[0]
    if ion_q.shape[0] != n_ion or wc_q.shape[0] != n_wc:
        raise ValueError("charge and position counts differ")
    cfg = _lib.Config()
    lib.dplr_lr_config_default(ctypes.byref(cfg))
    cfg.mesh[:] = [int(m) for m in mesh]
    cfg.order, cfg.beta, cfg.coulomb_k = int(order), float(beta), float(coulomb_k)
    cfg.precision = _lib.FP64 if dt == torch.float64 else _lib.FP32
    cfg.alias_range, cfg.flags = int(alias_range), int(flags)
    if ion_force is None:
        ion_force = torch.empty((n_ion, 3), dtype=dt, device=dev)
    if wc_force is None:
        wc_force = torch.empty((n_wc, 3), dtype=dt, device=dev)
    if energy is None:
        energy = torch.empty((), dtype=torch.float64, device=dev)
    if virial is None:
        virial = torch.empty(6, dtype=torch.float64, device=dev)
    boxa = (ctypes.c_double * 3)(*[float(b) for b in box])
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(lib.dplr_lr_compute_noalloc(
            ctypes.byref(cfg), boxa, n_ion, _ptr(ion_pos), _ptr(ion_q), n_wc, _ptr(wc_pos), _ptr(wc_q),
            _ptr(ion_force), _ptr(wc_force), ctypes.c_void_p(energy.data_ptr()),
            ctypes.c_void_p(virial.data_ptr()), ctypes.c_void_p(stream)))
    return energy, ion_force, wc_force, virial
