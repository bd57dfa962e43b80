"""kct: Krylov cone-beam CT reconstruction on MI355X (gfx950).

Python binding of the C ABI in ``include/kct.h``.  PyTorch provides device
memory and streams; every step of the method (forward projection, matched
back projection, the fused vector updates and the FP64 Krylov recurrences)
runs in the HIP kernels of ``libkct.so``.  There is no CPU fallback: if the
library or a GPU is missing, calls raise.

Layouts: volumes are (nz, ny, nx) tensors, projections (n_angles, nv, nu).
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import (KCT_BF16, KCT_CGLS, KCT_F16, KCT_F32, KCT_HIST_COLS, KCT_HYBRID_LSQR, KCT_IRN_TV_CGLS,
                   KCT_LSMR, KCT_LSQR, KctError)

__all__ = ["Geometry", "Plan", "State", "SOLVERS", "require_gpu", "KctError", "dtype_code", "library_path"]

SOLVERS = {"cgls": KCT_CGLS, "lsqr": KCT_LSQR, "lsmr": KCT_LSMR, "hybrid_lsqr": KCT_HYBRID_LSQR,
           "irn_tv_cgls": KCT_IRN_TV_CGLS, "ab_gmres": _lib.KCT_AB_GMRES, "ba_gmres": _lib.KCT_BA_GMRES,
           "sirt": _lib.KCT_SIRT, "os_sart": _lib.KCT_OS_SART, "hybrid_flsqr_tv": _lib.KCT_HYBRID_FLSQR_TV}
_DT = {torch.float32: KCT_F32, torch.bfloat16: KCT_BF16, torch.float16: KCT_F16}


def dtype_code(dt: torch.dtype) -> int:
    if dt not in _DT:
        raise TypeError(f"unsupported storage dtype {dt}")
    return _DT[dt]


def library_path() -> str:
    return _lib.LIB_PATH


def require_gpu():
    """Load the HIP library and check that a GPU is visible; raise otherwise."""
    _lib.load()
    if not torch.cuda.is_available():
        raise RuntimeError("kct needs a ROCm GPU (torch.cuda.is_available() is False)")


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Circular cone-beam geometry (mm, radians); see include/kct.h."""

    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    nu: int
    nv: int
    du: float
    dv: float
    dso: float
    dsd: float
    angles: tuple
    ox: float = 0.0
    oy: float = 0.0
    oz: float = 0.0

    @staticmethod
    def from_dict(d: dict) -> "Geometry":
        keys = {f.name for f in dataclasses.fields(Geometry)}
        kw = {k: d[k] for k in keys if k in d}
        kw["angles"] = tuple(float(a) for a in d["angles"])
        return Geometry(**kw)

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (len(self.angles), self.nv, self.nu)

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_rays(self) -> int:
        return len(self.angles) * self.nu * self.nv


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


LAMBDA_RULES = {"fixed": _lib.KCT_LAMBDA_FIXED, "gcv": _lib.KCT_LAMBDA_GCV, "dp": _lib.KCT_LAMBDA_DP}


BACKPROJECTORS = {"matched": _lib.KCT_BP_MATCHED, "interp": _lib.KCT_BP_INTERP}


def _params(solver, n_iter, lam, vec_dtype, tv_outer=0, tv_inner=0, tv_eps=1e-3, lam_rule="fixed",
            noise_level=0.0, backprojector="matched", n_subsets=0, stop_on_residual_increase=False,
            explicit_residual=False, warm_start=False):
    code = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    rule = LAMBDA_RULES[lam_rule] if isinstance(lam_rule, str) else int(lam_rule)
    bp = BACKPROJECTORS[backprojector] if isinstance(backprojector, str) else int(backprojector)
    flags = ((_lib.KCT_FLAG_STOP_ON_RESIDUAL_INCREASE if stop_on_residual_increase else 0)
             | (_lib.KCT_FLAG_EXPLICIT_RESIDUAL if explicit_residual else 0)
             | (_lib.KCT_FLAG_X0_GIVEN if warm_start else 0))
    return _lib.KctSolveParams(code, int(n_iter), float(lam), int(tv_outer), int(tv_inner), float(tv_eps),
                               dtype_code(vec_dtype), rule, float(noise_level), bp, int(n_subsets), flags, 0)


class Plan:
    """A geometry bound to one GPU: per-angle FP64 tables on the device."""

    def __init__(self, geom: Geometry, device: int = 0):
        require_gpu()
        self.geom = geom
        self.device = torch.device("cuda", device)
        self._angles = np.ascontiguousarray(np.asarray(geom.angles, dtype=np.float64))
        cg = _lib.KctGeometry(geom.nx, geom.ny, geom.nz, geom.vx, geom.vy, geom.vz, geom.ox, geom.oy, geom.oz,
                              geom.nu, geom.nv, geom.du, geom.dv, geom.dso, geom.dsd, len(self._angles),
                              self._angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_plan_create(ctypes.byref(cg), device, ctypes.byref(h)), "kct_plan_create")
        self._h = h
        self._reserved = set()  # volume storage types kct_plan_reserve was called for

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().kct_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def reserve(self, vol_dtype=torch.float32):
        """Allocate the padded volume copies that ``forward`` reads for volumes
        stored in ``vol_dtype`` (kct_plan_reserve; synchronous, once)."""
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_plan_reserve(self._h, dtype_code(vol_dtype)), "kct_plan_reserve")

    def check(self, stream=None):
        """Wait for ``stream`` and raise KctError if a back projection since the
        last check met a footprint beyond the plan's bounds (kct_plan_check)."""
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_plan_check(self._h, _stream_ptr(stream)), "kct_plan_check")

    def bwd_shape(self) -> dict:
        """The back projector's launch shape this plan chose (test hooks)."""
        kz, nc, pw, ph, split, rays = (ctypes.c_int() for _ in range(6))
        lib = _lib.load()
        lib.kct_debug_bwd_shape(self._h, ctypes.byref(kz), ctypes.byref(nc), ctypes.byref(pw), ctypes.byref(ph))
        lib.kct_debug_bwd_mode(self._h, ctypes.byref(split), ctypes.byref(rays))
        return dict(kz=kz.value, ncmax=nc.value, pw=pw.value, ph=ph.value, split=split.value, rays=rays.value)

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        _lib.check(_lib.load().kct_plan_device_bytes(self._h, ctypes.byref(n)), "kct_plan_device_bytes")
        return n.value

    # -- operators --------------------------------------------------------
    def _check(self, t: torch.Tensor, shape, what):
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{what} must be a tensor on {self.device}")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{what} must be a contiguous tensor of shape {tuple(shape)}")

    def forward(self, vol: torch.Tensor, out: torch.Tensor | None = None, out_dtype=None, stream=None):
        """A vol: ray sums, (n_angles, nv, nu)."""
        self._check(vol, self.geom.vol_shape, "volume")
        if out is None:
            out = torch.empty(self.geom.proj_shape, dtype=out_dtype or vol.dtype, device=self.device)
        self._check(out, self.geom.proj_shape, "projections")
        if vol.dtype not in self._reserved:
            self.reserve(vol.dtype)
            self._reserved.add(vol.dtype)
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_forward(self._h, ctypes.c_void_p(vol.data_ptr()), dtype_code(vol.dtype),
                                               ctypes.c_void_p(out.data_ptr()), dtype_code(out.dtype),
                                               _stream_ptr(stream)), "kct_forward")
        return out

    def forward_noalloc(self, vol: torch.Tensor, out: torch.Tensor, stream=None):
        """A vol into ``out`` through kct_forward_noalloc: the library allocates
        nothing (its padded copies live in a static device array of
        KCT_NOALLOC_SCRATCH_BYTES shared by every call on the GPU)."""
        self._check(vol, self.geom.vol_shape, "volume")
        self._check(out, self.geom.proj_shape, "projections")
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_forward_noalloc(self._h, ctypes.c_void_p(vol.data_ptr()), dtype_code(vol.dtype),
                                                       ctypes.c_void_p(out.data_ptr()), dtype_code(out.dtype),
                                                       _stream_ptr(stream)), "kct_forward_noalloc")
        return out

    def backproject(self, proj: torch.Tensor, out: torch.Tensor | None = None, out_dtype=None, stream=None):
        """A^T proj: matched back projection, (nz, ny, nx)."""
        self._check(proj, self.geom.proj_shape, "projections")
        if out is None:
            out = torch.empty(self.geom.vol_shape, dtype=out_dtype or proj.dtype, device=self.device)
        self._check(out, self.geom.vol_shape, "volume")
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_backproject(self._h, ctypes.c_void_p(proj.data_ptr()), dtype_code(proj.dtype),
                                                   ctypes.c_void_p(out.data_ptr()), dtype_code(out.dtype),
                                                   _stream_ptr(stream)), "kct_backproject")
        return out

    def backproject_interp(self, proj: torch.Tensor, out: torch.Tensor | None = None, out_dtype=None, stream=None):
        """B proj: the unmatched, voxel-driven interpolating back projection, (nz, ny, nx)."""
        self._check(proj, self.geom.proj_shape, "projections")
        if out is None:
            out = torch.empty(self.geom.vol_shape, dtype=out_dtype or proj.dtype, device=self.device)
        self._check(out, self.geom.vol_shape, "volume")
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_backproject_interp(self._h, ctypes.c_void_p(proj.data_ptr()),
                                                          dtype_code(proj.dtype), ctypes.c_void_p(out.data_ptr()),
                                                          dtype_code(out.dtype), _stream_ptr(stream)),
                       "kct_backproject_interp")
        return out

    # -- solvers ----------------------------------------------------------
    def workspace_bytes(self, solver="cgls", n_iter=20, lam=0.0, vec_dtype=torch.float32, **tv) -> int:
        p = _params(solver, n_iter, lam, vec_dtype, **tv)
        n = ctypes.c_size_t()
        _lib.check(_lib.load().kct_solve_workspace_bytes(self._h, ctypes.byref(p), ctypes.byref(n)),
                   "kct_solve_workspace_bytes")
        return n.value

    def history_rows(self, solver, n_iter, tv_outer=0, tv_inner=0) -> int:
        code = SOLVERS[solver] if isinstance(solver, str) else int(solver)
        return tv_outer * tv_inner if code == KCT_IRN_TV_CGLS else n_iter

    def solve(self, b: torch.Tensor, solver="cgls", n_iter=20, lam=0.0, vec_dtype=torch.float32,
              x: torch.Tensor | None = None, workspace: torch.Tensor | None = None, history: bool = True,
              stream=None, **tv):
        """Run `solver` from x0 = 0 for `n_iter` iterations.  Returns (x, history).

        Keyword options: tv_outer, tv_inner, tv_eps (IRN-TV; fLSQR-TV takes
        tv_inner = CG steps per pseudoinverse and tv_eps); lam_rule
        ("fixed", "gcv" or "dp") and noise_level (hybrid LSQR, fLSQR-TV); backprojector
        ("matched" or "interp", AB-/BA-GMRES); n_subsets (OS-SART; lam is
        the relaxation of SIRT and OS-SART); stop_on_residual_increase and
        explicit_residual (CGLS, LSQR, LSMR); warm_start (x holds x0: CGLS,
        undamped LSQR/LSMR, SIRT, OS-SART).  history is an
        (n_rows, KCT_HIST_COLS) float64 device tensor or None.  The call only
        enqueues work on the stream.
        """
        self._check(b, self.geom.proj_shape, "b")
        if b.dtype != torch.float32:
            raise TypeError("b must be float32")
        if x is None:
            if tv.get("warm_start"):
                raise ValueError("warm_start needs x (it holds x0)")
            x = torch.empty(self.geom.vol_shape, dtype=torch.float32, device=self.device)
        self._check(x, self.geom.vol_shape, "x")
        p = _params(solver, n_iter, lam, vec_dtype, **tv)
        need = self.workspace_bytes(solver, n_iter, lam, vec_dtype, **tv)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        hist = None
        if history:
            rows = self.history_rows(solver, n_iter, tv.get("tv_outer", 0), tv.get("tv_inner", 0))
            hist = torch.zeros((max(rows, 1), KCT_HIST_COLS), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_solve(self._h, ctypes.byref(p), ctypes.c_void_p(b.data_ptr()),
                                             ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                                             workspace.numel(),
                                             ctypes.c_void_p(hist.data_ptr() if hist is not None else 0),
                                             _stream_ptr(stream)), "kct_solve")
        return x, hist

    def state(self, b, solver="cgls", n_iter=20, lam=0.0, vec_dtype=torch.float32, stream=None, **tv) -> "State":
        return State(self, b, solver, n_iter, lam, vec_dtype, stream, **tv)

    def resume_state(self, b, checkpoint: dict, stream=None) -> "State":
        """A State continuing a run from ``State.checkpoint()`` (same geometry, same b)."""
        c = checkpoint
        return State(self, b, c["solver"], c["n_iter"], c["lam"], c["vec_dtype"], stream, _resume=c, **c["options"])


class State:
    """Iteration-level solver run (kct_state_*), owning its buffers as tensors."""

    def __init__(self, plan: Plan, b, solver, n_iter, lam, vec_dtype, stream=None, _resume=None, **tv):
        plan._check(b, plan.geom.proj_shape, "b")
        self.plan = plan
        self.b = b
        self.n_iter = n_iter
        self._args = dict(solver=solver, n_iter=n_iter, lam=lam, vec_dtype=vec_dtype, options=dict(tv))
        self.stream = stream if stream is not None else torch.cuda.current_stream(plan.device)
        need = plan.workspace_bytes(solver, n_iter, lam, vec_dtype, **tv)
        rows = plan.history_rows(solver, n_iter, tv.get("tv_outer", 0), tv.get("tv_inner", 0))
        # Allocated (and the history zeroed) on the run's stream, ordered
        # before its kernels.
        with torch.cuda.stream(self.stream):
            self.x = torch.empty(plan.geom.vol_shape, dtype=torch.float32, device=plan.device)
            self.workspace = torch.empty(need, dtype=torch.uint8, device=plan.device)
            self.history = torch.zeros((max(rows, 1), KCT_HIST_COLS), dtype=torch.float64, device=plan.device)
        p = _params(solver, n_iter, lam, vec_dtype, **tv)
        h = ctypes.c_void_p()
        args = (plan.handle, ctypes.byref(p), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(self.x.data_ptr()),
                ctypes.c_void_p(self.workspace.data_ptr()), need, ctypes.c_void_p(self.history.data_ptr()),
                ctypes.c_void_p(self.stream.cuda_stream))
        if _resume is None:
            _lib.check(_lib.load().kct_state_create(*args, ctypes.byref(h)), "kct_state_create")
        else:
            if _resume["workspace"].numel() != need or _resume["history"].shape != self.history.shape:
                raise ValueError("checkpoint does not match this run's buffer sizes")
            with torch.cuda.stream(self.stream):
                self.workspace.copy_(_resume["workspace"])
                self.x.copy_(_resume["x"])
                self.history.copy_(_resume["history"])
            _lib.check(_lib.load().kct_state_resume(*args, int(_resume["iters"]), ctypes.byref(h)),
                       "kct_state_resume")
        self._h = h

    def checkpoint(self) -> dict:
        """Host copy of the run's whole state (workspace, x, history) and its
        arguments; waits for the stream.  ``Plan.resume_state`` continues it."""
        self.step(0)  # the initialisation, if it has not been enqueued yet
        self.stream.synchronize()
        it, _ = self.progress()
        return dict(self._args, iters=it, workspace=self.workspace.cpu(), x=self.x.cpu(),
                    history=self.history.cpu())

    def step(self, n: int = 1):
        with torch.cuda.device(self.plan.device):
            _lib.check(_lib.load().kct_state_step(self._h, int(n)), "kct_state_step")

    def progress(self):
        it, fin = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.load().kct_state_progress(self._h, ctypes.byref(it), ctypes.byref(fin)),
                   "kct_state_progress")
        return it.value, bool(fin.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().kct_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
