"""Learned coarse-mesh form: coarse-mesh PPPM plus a per-particle network
correction, with the fine mesh as fallback.

Argument marshalling and orchestration only: the descriptor, the network
(BF16 MFMA), its backward, the optimiser and both PPPM plans run in
libdplr_lr's kernels.  Training targets are fine-minus-coarse PPPM force
residuals computed by the library's own plans on seeded, spacing-matched
training boxes.
"""
from __future__ import annotations

import ctypes
import dataclasses
import json
import math
from typing import Optional

import numpy as np
import torch

from . import _lib
from .plan import Plan, _ptr

N_IN, N_H, N_OUT = 128, 64, 32
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H, N_H)),
          ("b3", (N_H,)), ("W4", (N_H, N_OUT)), ("b4", (N_OUT,)), ("mu", (N_IN,)), ("inv_sigma", (N_IN,))]
N_TRAIN = sum(int(np.prod(s)) for k, s in SHAPES if k not in ("mu", "inv_sigma"))


def pack(params: dict) -> np.ndarray:
    """Packed FP32 parameter vector in the C ABI's order."""
    out = [np.asarray(params[k], dtype=np.float32).reshape(-1) for k, _ in SHAPES]
    return np.concatenate(out)


def unpack(vec) -> dict:
    vec = np.asarray(vec, dtype=np.float32)
    out, o = {}, 0
    for k, s in SHAPES:
        n = int(np.prod(s))
        out[k] = vec[o:o + n].reshape(s).copy()
        o += n
    return out


def init_params(seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    p = {}
    for l, (a, b) in enumerate([(N_IN, N_H), (N_H, N_H), (N_H, N_H), (N_H, N_OUT)], start=1):
        p[f"W{l}"] = rng.normal(0.0, 1.0 / math.sqrt(a), (a, b))
        p[f"b{l}"] = np.zeros(b)
    p["W4"] *= 0.1
    p["mu"] = np.zeros(N_IN)
    p["inv_sigma"] = np.ones(N_IN)
    return p


class Mlp:
    """The correction network (libdplr_lr dplr_lr_mlp_*)."""

    def __init__(self, capacity: int, cutoff: float = 4.0, out_scale: float = 0.01,
                 device: Optional[torch.device] = None):
        lib = _lib.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        cfg = _lib.MlpConfig()
        lib.dplr_lr_mlp_config_default(ctypes.byref(cfg))
        cfg.cutoff, cfg.out_scale, cfg.capacity = float(cutoff), float(out_scale), int(capacity)
        self.cfg = cfg
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            s = torch.cuda.current_stream(self.device).cuda_stream
            _lib.check_mlp(lib.dplr_lr_mlp_create(ctypes.byref(cfg), ctypes.c_void_p(s), ctypes.byref(h)))
        self._h = h
        self.n_params = int(lib.dplr_lr_mlp_param_count())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().dplr_lr_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check_mlp(_lib.load().dplr_lr_mlp_set_stream(self._h, ctypes.c_void_p(s)), self._h)

    def set_params(self, params):
        vec = pack(params) if isinstance(params, dict) else np.ascontiguousarray(params, dtype=np.float32)
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_set_params(self._h, vec.ctypes.data_as(ctypes.c_void_p),
                                                                vec.size), self._h)

    def get_params(self) -> dict:
        vec = np.zeros(self.n_params, dtype=np.float32)
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_get_params(self._h, vec.ctypes.data_as(ctypes.c_void_p),
                                                                vec.size), self._h)
        return unpack(vec)

    def get_state(self) -> np.ndarray:
        """The whole training state (parameters, Adam moments and step count,
        normalisation sums, training charges) as a uint8 array."""
        lib = _lib.load()
        blob = np.zeros(int(lib.dplr_lr_mlp_state_bytes()), dtype=np.uint8)
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(lib.dplr_lr_mlp_get_state(self._h, blob.ctypes.data_as(ctypes.c_void_p), blob.size),
                           self._h)
        return blob

    def set_state(self, blob):
        """Restores a state from get_state (training then continues bitwise
        as it would have)."""
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_set_state(self._h, blob.ctypes.data_as(ctypes.c_void_p),
                                                               blob.size), self._h)

    @staticmethod
    def _box(box):
        return (ctypes.c_double * 3)(*[float(b) for b in box])

    def forward(self, box, ion_pos, ion_q, wc_pos, wc_q, ion_dF=None, wc_dF=None, accumulate=False):
        n_ion, n_wc = ion_pos.shape[0], wc_pos.shape[0]
        if ion_dF is None:
            ion_dF = torch.empty((n_ion, 3), dtype=torch.float32, device=self.device)
        if wc_dF is None:
            wc_dF = torch.empty((n_wc, 3), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_forward(
                self._h, self._box(box), n_ion, _ptr(ion_pos), _ptr(ion_q), n_wc, _ptr(wc_pos), _ptr(wc_q),
                _ptr(ion_dF), _ptr(wc_dF), 1 if accumulate else 0), self._h)
        return ion_dF, wc_dF

    def train_step(self, box, ion_pos, ion_q, wc_pos, wc_q, ion_tgt, wc_tgt, lr: float, want_grad=False,
                   ion_base=None, wc_base=None):
        """One training step; with ion_base / wc_base the targets are
        target - base (the residual is formed in the kernel)."""
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        grad = torch.empty(N_TRAIN, dtype=torch.float32, device=self.device) if want_grad else None
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_train_step(
                self._h, self._box(box), ion_pos.shape[0], _ptr(ion_pos), _ptr(ion_q), wc_pos.shape[0],
                _ptr(wc_pos), _ptr(wc_q), _ptr(ion_tgt), _ptr(wc_tgt), _ptr(ion_base), _ptr(wc_base),
                ctypes.c_float(lr), ctypes.c_void_p(loss.data_ptr()), _ptr(grad)), self._h)
        return loss, grad

    def norm_accumulate(self, box, ion_pos, ion_q, wc_pos, wc_q):
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_norm_accumulate(
                self._h, self._box(box), ion_pos.shape[0], _ptr(ion_pos), _ptr(ion_q), wc_pos.shape[0],
                _ptr(wc_pos), _ptr(wc_q)), self._h)

    def norm_finish(self):
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_norm_finish(self._h), self._h)

    def set_train_charges(self, charges):
        arr = np.ascontiguousarray(charges, dtype=np.float32)
        _lib.check_mlp(_lib.load().dplr_lr_mlp_set_train_charges(self._h, arr.ctypes.data_as(ctypes.c_void_p),
                                                                  int(arr.size)), self._h)

    def check_charges(self, ion_q, wc_q):
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_check_charges(self._h, ion_q.shape[0], _ptr(ion_q),
                                                                  wc_q.shape[0], _ptr(wc_q)), self._h)

    def audit(self, ion_f, ion_ref, wc_f, wc_ref, accumulate=False):
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_audit(
                self._h, ion_f.shape[0], _ptr(ion_f), _ptr(ion_ref), wc_f.shape[0], _ptr(wc_f), _ptr(wc_ref),
                1 if accumulate else 0), self._h)

    def read_stats(self) -> dict:
        """Guard statistics recorded on the device (synchronises the stream)."""
        st = _lib.GuardStats()
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_read_stats(self._h, ctypes.byref(st)), self._h)
        return {k: getattr(st, k) for k, _ in _lib.GuardStats._fields_}

    def descriptor(self, box, ion_pos, ion_q, wc_pos, wc_q):
        n = ion_pos.shape[0] + wc_pos.shape[0]
        T = torch.empty((n, 32, 4), dtype=torch.float32, device=self.device)
        order = torch.empty(n, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            self._bind()
            _lib.check_mlp(_lib.load().dplr_lr_mlp_descriptor(
                self._h, self._box(box), ion_pos.shape[0], _ptr(ion_pos), _ptr(ion_q), wc_pos.shape[0],
                _ptr(wc_pos), _ptr(wc_q), _ptr(T), _ptr(order)), self._h)
        return T, order


def guard_decide(cfg: dict, stats: dict) -> int:
    """Host-side fallback decision (dplr_lr_guard_decide)."""
    c = _lib.GuardConfig(**cfg)
    s = _lib.GuardStats(**stats)
    d = ctypes.c_int32()
    _lib.check_mlp(_lib.load().dplr_lr_guard_decide(ctypes.byref(c), ctypes.byref(s), ctypes.byref(d)))
    return int(d.value)


@dataclasses.dataclass
class TrainReport:
    losses: list
    heldout_rel_rmse_learned: float
    heldout_rel_rmse_coarse: float
    boxes: int
    epochs: int


def _dev_tensors(sys, device):
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=device)
    return t(sys.ion_pos), t(sys.ion_q), t(sys.wc_pos), t(sys.wc_q)


def plan_forces(sys, coarse: Plan, fine: Plan, device):
    """Device inputs of one system and the coarse- and fine-mesh PPPM forces
    of the library's plans (the residual is formed by the training kernel)."""
    ri, qi, rw, qw = _dev_tensors(sys, device)
    _, fci, fcw, _ = coarse.compute(ri, qi, rw, qw)
    fci, fcw = fci.clone(), fcw.clone()
    _, ffi, ffw, _ = fine.compute(ri, qi, rw, qw)
    return (ri, qi, rw, qw), (fci, fcw), (ffi.clone(), ffw.clone())


def train(boxes, heldout, coarse_mesh: int, fine_mesh: int, coarse_order: int = 5, fine_order: int = 8,
          epochs: int = 4, lr: float = 2e-3, seed: int = 0, mlp: Optional[Mlp] = None,
          device: Optional[torch.device] = None, log=None, checkpoint: Optional[str] = None,
          resume: Optional[str] = None, stop_after: Optional[int] = None) -> tuple:
    """Train the correction on seeded boxes (list of systems.System, same box).
    Returns (mlp, TrainReport).

    checkpoint: path of a .npz file rewritten at the end of every epoch with
    the network's training state (parameters, Adam moments and step count,
    normalisation), the epoch and step counters, the losses so far and the
    state of the generator that orders the boxes.  resume: such a file to
    continue from, with the same boxes, epochs, lr and seed; the result is
    bitwise that of an uninterrupted run.  stop_after: run at most this many
    epochs in this call (a time slice of a longer run)."""
    device = torch.device(device) if device is not None else torch.device("cuda", 0)
    box = boxes[0].box
    cap = max(s.n for s in list(boxes) + list(heldout))
    coarse = Plan(coarse_mesh, order=coarse_order, precision="fp32", capacity=cap, device=device)
    fine = Plan(fine_mesh, order=fine_order, precision="fp32", capacity=cap, device=device)
    coarse.set_box(box)
    fine.set_box(box)
    if mlp is None:
        mlp = Mlp(cap, device=device)
    data = [plan_forces(s, coarse, fine, device) for s in boxes]
    nsteps = epochs * len(data)
    rng = np.random.default_rng(seed)
    run = dict(seed=seed, epochs=epochs, lr=lr, nboxes=len(data))
    if resume is not None:
        with np.load(resume, allow_pickle=False) as ck:
            for k, v in run.items():
                if type(v)(ck[k]) != v:
                    raise ValueError(f"checkpoint {resume} is from a run with {k}={ck[k]}, not {v}")
            mlp.set_state(ck["mlp_state"])
            ep0, step = int(ck["epoch"]), int(ck["step"])
            rng.bit_generator.state = json.loads(str(ck["rng_state"]))
            losses = [float(x) for x in ck["losses"]]
    else:
        mlp.set_params(init_params(seed))
        # input normalisation from the training descriptors (device sums)
        for (ri, qi, rw, qw), _, _ in data[: min(len(data), 64)]:
            mlp.norm_accumulate(box, ri, qi, rw, qw)
        mlp.norm_finish()
        ep0, step, losses = 0, 0, []
    ep1 = epochs if stop_after is None else min(epochs, ep0 + int(stop_after))
    for ep in range(ep0, ep1):
        ep_losses = []
        for i in rng.permutation(len(data)):
            (ri, qi, rw, qw), (fci, fcw), (ffi, ffw) = data[i]
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * step / max(1, nsteps)))
            loss, _ = mlp.train_step(box, ri, qi, rw, qw, ffi, ffw, lr_t, ion_base=fci, wc_base=fcw)
            ep_losses.append(loss)
            step += 1
        losses += [float(x) for x in ep_losses]
        if log:
            log(f"epoch {ep}: mean loss {float(np.mean(losses[-len(data):])):.4e}")
        if checkpoint is not None:
            with open(checkpoint, "wb") as f:
                np.savez(f, mlp_state=mlp.get_state(), epoch=ep + 1, step=step,
                         rng_state=json.dumps(rng.bit_generator.state), losses=np.asarray(losses), **run)
    # held-out relative force error against the fine mesh: the coarse forces
    # alone, then with the correction (audit sums accumulated over the boxes)
    held = [plan_forces(s, coarse, fine, device) for s in heldout]
    for k, ((ri, qi, rw, qw), (fci, fcw), (ffi, ffw)) in enumerate(held):
        mlp.audit(fci, ffi, fcw, ffw, accumulate=k > 0)
    rel_coarse = mlp.read_stats()["audit_rel_rmse"]
    for k, ((ri, qi, rw, qw), (fci, fcw), (ffi, ffw)) in enumerate(held):
        mlp.forward(box, ri, qi, rw, qw, fci, fcw, accumulate=True)
        mlp.audit(fci, ffi, fcw, ffw, accumulate=k > 0)
    rel_learned = mlp.read_stats()["audit_rel_rmse"]
    rep = TrainReport(losses, rel_learned, rel_coarse, len(boxes), epochs)
    coarse.close()
    fine.close()
    return mlp, rep


class LearnedCoarse:
    """Coarse-mesh PPPM + network correction, with a guarded fallback to the
    fine mesh.  compute() returns (E, F_ion, F_wc, virial, mode) where mode is
    'learned', 'fine' or 'audit'.  Energy and virial come from the coarse plan
    in the learned mode (the network corrects forces only).  Every statistic
    the guard uses is measured on the device (charge check, forward, audit);
    this class only carries the step counter and the decision."""

    def __init__(self, box, coarse: Plan, fine: Plan, mlp: Mlp, guard_cfg: Optional[dict] = None,
                 train_charges=(6.0, 1.0, -8.0)):
        if coarse.precision != "fp32":
            raise ValueError("the correction adds FP32 forces: the coarse plan must be fp32")
        self.box = tuple(float(b) for b in box)
        self.coarse, self.fine, self.mlp = coarse, fine, mlp
        self.guard_cfg = dict(max_audit_rel_rmse=1e-3, max_correction_ratio=0.5, audit_interval=100,
                              min_neighbours=0.0, max_neighbours=0.0)
        if guard_cfg:
            self.guard_cfg.update(guard_cfg)
        mlp.set_train_charges(train_charges)
        self.steps_since_audit = 0
        self.audited = False
        self.stats = {}
        self.force_fine = False

    def _learned(self, ri, qi, rw, qw):
        E, fi, fw, W = self.coarse.compute(ri, qi, rw, qw)
        self.mlp.forward(self.box, ri, qi, rw, qw, fi, fw, accumulate=True)
        return E, fi, fw, W

    def compute(self, ion_pos, ion_q, wc_pos, wc_q):
        self.mlp.check_charges(ion_q, wc_q)
        st = self.mlp.read_stats()
        st["steps_since_audit"] = self.steps_since_audit
        st["audit_valid"] = 1 if self.audited else 0
        self.stats = st
        d = _lib.GUARD_FINE if self.force_fine else guard_decide(self.guard_cfg, st)
        if d == _lib.GUARD_FINE:
            E, fi, fw, W = self.fine.compute(ion_pos, ion_q, wc_pos, wc_q)
            return E, fi, fw, W, "fine"
        if d == _lib.GUARD_AUDIT:
            Ef, ffi, ffw, Wf = [x.clone() for x in self.fine.compute(ion_pos, ion_q, wc_pos, wc_q)]
            E, fi, fw, W = self._learned(ion_pos, ion_q, wc_pos, wc_q)
            self.mlp.audit(fi, ffi, fw, ffw)
            self.audited = True
            self.steps_since_audit = 0
            self.stats = self.mlp.read_stats()
            # the audit's fine result is the one returned
            return Ef, ffi, ffw, Wf, "audit"
        self.steps_since_audit += 1
        E, fi, fw, W = self._learned(ion_pos, ion_q, wc_pos, wc_q)
        return E, fi, fw, W, "learned"
