"""Brute-force dense system matrix for tiny grids (NumPy, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

An independent formulation of the same operator as ``projector.py``: instead
of walking each ray through the merged plane crossings, every (ray, voxel)
pair is intersected directly, by clipping the ray parameter against the
voxel's three slabs.  Ray end points are built by rotating the detector frame
rather than by the explicit formulas used in ``siddon.c``.  Agreement of the
two, on grids small enough to enumerate every pair, pins the traversal.
"""
from __future__ import annotations

import numpy as np

from .projector import Geometry


def ray_endpoints(g: Geometry):
    """Source and pixel-centre positions, each of shape (na, nv, nu, 3).

    In the frame that rotates with the gantry the source sits at (DSO, 0, 0)
    and the detector plane at x = DSO - DSD, with the u axis along +y and v
    along +z.  Rotating that frame by the angle about z gives the lab frame.
    """
    ang = np.asarray(g.angles, dtype=np.float64)
    na = ang.size
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv
    local = np.zeros((g.nv, g.nu, 3))
    local[..., 0] = g.dso - g.dsd
    local[..., 1] = u[None, :]
    local[..., 2] = v[:, None]
    src = np.zeros((na, g.nv, g.nu, 3))
    pix = np.zeros((na, g.nv, g.nu, 3))
    for a in range(na):
        c, s = np.cos(ang[a]), np.sin(ang[a])
        R = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
        pix[a] = local @ R.T
        src[a] = R @ np.array([g.dso, 0.0, 0.0])
    return src, pix


def _slab_intervals(p0, d, lo, h, n):
    """Per-voxel parameter interval along one axis: arrays (n,) of t_lo, t_hi.

    With d == 0 the ray is inside the half-open slab [lo_i, lo_i + h) for all
    t, or for no t.
    """
    edges = lo + h * np.arange(n + 1)
    if d != 0.0:
        t = (edges - p0) / d
        return np.minimum(t[:-1], t[1:]), np.maximum(t[:-1], t[1:])
    inside = (edges[:-1] <= p0) & (p0 < edges[1:])
    t_lo = np.where(inside, -np.inf, np.inf)
    t_hi = np.where(inside, np.inf, -np.inf)
    return t_lo, t_hi


def system_matrix(g: Geometry) -> np.ndarray:
    """Dense A of shape (na*nv*nu, nz*ny*nx); entry = mm of ray inside voxel."""
    src, pix = ray_endpoints(g)
    X0 = g.ox - 0.5 * g.nx * g.vx
    Y0 = g.oy - 0.5 * g.ny * g.vy
    Z0 = g.oz - 0.5 * g.nz * g.vz
    na = len(g.angles)
    A = np.zeros((na * g.nv * g.nu, g.nz * g.ny * g.nx))
    r = 0
    for a in range(na):
        for iv in range(g.nv):
            for iu in range(g.nu):
                p0 = src[a, iv, iu]
                d = pix[a, iv, iu] - p0
                xl, xh = _slab_intervals(p0[0], d[0], X0, g.vx, g.nx)
                yl, yh = _slab_intervals(p0[1], d[1], Y0, g.vy, g.ny)
                zl, zh = _slab_intervals(p0[2], d[2], Z0, g.vz, g.nz)
                lo = np.maximum(np.maximum(zl[:, None, None], yl[None, :, None]), xl[None, None, :])
                hi = np.minimum(np.minimum(zh[:, None, None], yh[None, :, None]), xh[None, None, :])
                lo = np.maximum(lo, 0.0)
                hi = np.minimum(hi, 1.0)
                A[r] = (np.maximum(hi - lo, 0.0) * np.linalg.norm(d)).ravel()
                r += 1
    return A


def box_chords(g: Geometry, lo=None, hi=None) -> np.ndarray:
    """Closed-form chord length (mm) of every ray through an axis-aligned box.

    Defaults to the whole volume box.  Shape (na, nv, nu).
    """
    src, pix = ray_endpoints(g)
    if lo is None:
        lo = (g.ox - 0.5 * g.nx * g.vx, g.oy - 0.5 * g.ny * g.vy, g.oz - 0.5 * g.nz * g.vz)
    if hi is None:
        hi = (g.ox + 0.5 * g.nx * g.vx, g.oy + 0.5 * g.ny * g.vy, g.oz + 0.5 * g.nz * g.vz)
    d = pix - src
    with np.errstate(divide="ignore", invalid="ignore"):
        t_in = np.zeros(d.shape[:-1])
        t_out = np.ones(d.shape[:-1])
        for ax in range(3):
            ta = (lo[ax] - src[..., ax]) / d[..., ax]
            tb = (hi[ax] - src[..., ax]) / d[..., ax]
            par = d[..., ax] == 0.0
            inside = (src[..., ax] >= lo[ax]) & (src[..., ax] < hi[ax])
            tmin = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(ta, tb))
            tmax = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(ta, tb))
            t_in = np.maximum(t_in, tmin)
            t_out = np.minimum(t_out, tmax)
    return np.maximum(t_out - t_in, 0.0) * np.linalg.norm(d, axis=-1)


def sphere_chords(g: Geometry, centre, radius) -> np.ndarray:
    """Closed-form chord 2 sqrt(R^2 - dist^2) of every ray through a ball."""
    src, pix = ray_endpoints(g)
    d = pix - src
    dn = np.linalg.norm(d, axis=-1, keepdims=True)
    e = d / dn
    w = np.asarray(centre, dtype=np.float64) - src
    along = np.sum(w * e, axis=-1, keepdims=True)
    perp2 = np.sum((w - along * e) ** 2, axis=-1)
    return 2.0 * np.sqrt(np.maximum(radius * radius - perp2, 0.0))
