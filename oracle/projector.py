"""FP64 Siddon projector of the oracle (ctypes wrapper around ``siddon.c``).

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the GPU library.

The operator is the system matrix A of A x + e = b (paper, Sec. 1, eq. (original_pbm)):
row i is ray i, column j is voxel j, and a_ij is the length (mm) of ray i
inside voxel j.  ``forward`` computes A x and ``adjoint`` computes A^T y by
scattering the same traced segments, so the pair is an exact transpose.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "siddon.c")
_LIB_PATH = os.path.join(_HERE, "_siddon.so")
_lock = threading.Lock()
_lib = None


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Circular cone-beam geometry.  Lengths in mm, angles in radians.

    Volume: nx*ny*nz voxels of size (vx, vy, vz), centred at (ox, oy, oz),
    stored x[k][j][i].  Flat detector of nu*nv pixels with pitch (du, dv);
    projections stored y[a][iv][iu].  Source-origin distance ``dso`` and
    source-detector distance ``dsd``.
    """

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

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (len(self.angles), self.nv, self.nu)

    @staticmethod
    def from_dict(d: dict) -> "Geometry":
        keys = {f.name for f in dataclasses.fields(Geometry)}
        kw = {k: d[k] for k in keys if k in d}
        kw["angles"] = tuple(float(a) for a in d["angles"])
        return Geometry(**kw)

    def with_angles(self, angles) -> "Geometry":
        return dataclasses.replace(self, angles=tuple(float(a) for a in angles))


class _CGeom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
        ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double),
        ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("dso", ctypes.c_double), ("dsd", ctypes.c_double),
        ("na", ctypes.c_int32),
        ("angles", ctypes.POINTER(ctypes.c_double)),
    ]


def build(force: bool = False) -> str:
    """Compile ``siddon.c`` into ``_siddon.so`` with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.POINTER
            lib.ora_forward.argtypes = [P(_CGeom), P(ctypes.c_double), P(ctypes.c_double)]
            lib.ora_adjoint.argtypes = [P(_CGeom), P(ctypes.c_double), P(ctypes.c_double)]
            lib.ora_ray_segments.argtypes = [P(_CGeom), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             P(ctypes.c_int64), P(ctypes.c_double), ctypes.c_int]
            lib.ora_forward_rays.argtypes = [P(_CGeom), P(ctypes.c_double), P(ctypes.c_int64),
                                             ctypes.c_int64, P(ctypes.c_double)]
            lib.ora_count_nnz.argtypes = [P(_CGeom), P(ctypes.c_int64), P(ctypes.c_int64)]
            lib.ora_num_threads.restype = ctypes.c_int
            lib.ora_set_num_threads.argtypes = [ctypes.c_int]
            _lib = lib
    return _lib


def _cgeom(g: Geometry):
    ang = np.ascontiguousarray(np.asarray(g.angles, dtype=np.float64))
    cg = _CGeom(g.nx, g.ny, g.nz, g.vx, g.vy, g.vz, g.ox, g.oy, g.oz,
                g.nu, g.nv, g.du, g.dv, g.dso, g.dsd, len(ang),
                ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return cg, ang  # keep `ang` alive with the struct


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def forward(g: Geometry, x) -> np.ndarray:
    """y = A x in FP64.  ``x`` has shape (nz, ny, nx); returns (na, nv, nu)."""
    lib = _load()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(g.vol_shape))
    y = np.empty(g.proj_shape, dtype=np.float64)
    cg, _keep = _cgeom(g)
    if lib.ora_forward(ctypes.byref(cg), _dptr(x), _dptr(y)) != 0:
        raise MemoryError("oracle forward: allocation failed")
    return y


def adjoint(g: Geometry, y) -> np.ndarray:
    """x = A^T y in FP64.  ``y`` has shape (na, nv, nu); returns (nz, ny, nx)."""
    lib = _load()
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(g.proj_shape))
    x = np.empty(g.vol_shape, dtype=np.float64)
    cg, _keep = _cgeom(g)
    if lib.ora_adjoint(ctypes.byref(cg), _dptr(y), _dptr(x)) != 0:
        raise MemoryError("oracle adjoint: allocation failed")
    return x


def forward_rays(g: Geometry, x, rays) -> np.ndarray:
    """(A x)_r for the flat ray ids ``rays`` (r = (a*nv + iv)*nu + iu)."""
    lib = _load()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(g.vol_shape))
    rays = np.ascontiguousarray(np.asarray(rays, dtype=np.int64).ravel())
    out = np.empty(rays.size, dtype=np.float64)
    cg, _keep = _cgeom(g)
    rc = lib.ora_forward_rays(ctypes.byref(cg), _dptr(x),
                              rays.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rays.size, _dptr(out))
    if rc != 0:
        raise MemoryError("oracle forward_rays: allocation failed")
    return out


def ray_segments(g: Geometry, a: int, iv: int, iu: int):
    """(voxel linear indices, lengths in mm) of the segments of one ray."""
    lib = _load()
    cap = 3 * (g.nx + g.ny + g.nz + 8)
    idx = np.empty(cap, dtype=np.int64)
    ln = np.empty(cap, dtype=np.float64)
    cg, _keep = _cgeom(g)
    n = lib.ora_ray_segments(ctypes.byref(cg), a, iv, iu,
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(ln), cap)
    if n < 0:
        raise RuntimeError("oracle ray_segments failed")
    return idx[:n].copy(), ln[:n].copy()


def count_nnz(g: Geometry):
    """(nonzero entries of A, rays that meet the volume) for geometry g."""
    lib = _load()
    nnz, hits = ctypes.c_int64(), ctypes.c_int64()
    cg, _keep = _cgeom(g)
    if lib.ora_count_nnz(ctypes.byref(cg), ctypes.byref(nnz), ctypes.byref(hits)) != 0:
        raise MemoryError("oracle count_nnz: allocation failed")
    return int(nnz.value), int(hits.value)


def num_threads() -> int:
    return int(_load().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for later projector calls.

    ``forward`` gives the same result for any count (each ray is summed by one
    thread).  ``adjoint`` sums one partial volume per thread, in thread order,
    so its result can change with the count at FP64 rounding level (about
    1e-16 relative)."""
    _load().ora_set_num_threads(int(n))
