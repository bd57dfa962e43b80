"""Unmatched back projector B of the oracle (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

GPU toolboxes back-project with an approximation B of A^T rather than with
the exact transpose (Sec. 2.1.4); AB- and BA-GMRES take such a B as a right or
left preconditioner.  This is the usual voxel-driven form: the centre p of
voxel j is projected onto the detector along the ray from the source, the
projection at that angle is interpolated bilinearly there (zero outside the
detector), and the value is weighted so that B approximates A^T on smooth
data:

  w = DSO - (p_x cos t + p_y sin t)          depth of p along the central ray
  u = DSD (-p_x sin t + p_y cos t) / w       detector coordinates of p's image
  v = DSD p_z / w
  weight = V / (du dv) * (DSD / w)^2 * |d| / DSD,   |d| = sqrt(DSD^2 + u^2 + v^2)

(V = vx vy vz.  Rays cross the voxel at a density of (DSD/w)^2 / (du dv cos g)
per unit area normal to them, cos g = DSD / |d|, and a bundle through the
voxel carries V per unit normal area, so sum_i a_ij y_i ~ weight * y(u, v).)
Pixel (iu, iv) sits at ((iu - (nu-1)/2) du, (iv - (nv-1)/2) dv), as in the
projector geometry.
"""
from __future__ import annotations

import numpy as np

from .projector import Geometry


def _centres(n, h, o):
    return o - n * h / 2.0 + (np.arange(n) + 0.5) * h


def _bilinear(img, fu, fv):
    """img[iv, iu] at fractional indices (fu, fv); 0 outside the pixel grid."""
    nv, nu = img.shape
    i0 = np.floor(fu).astype(np.int64)
    j0 = np.floor(fv).astype(np.int64)
    au, av = fu - i0, fv - j0
    out = np.zeros(np.broadcast(fu, fv).shape)
    for dj, wv in ((0, 1.0 - av), (1, av)):
        for di, wu in ((0, 1.0 - au), (1, au)):
            ii, jj = i0 + di, j0 + dj
            ok = (ii >= 0) & (ii < nu) & (jj >= 0) & (jj < nv)
            vals = np.where(ok, img[np.clip(jj, 0, nv - 1), np.clip(ii, 0, nu - 1)], 0.0)
            out += wu * wv * vals
    return out


def backproject_interp(g: Geometry, y) -> np.ndarray:
    """x = B y for projections ``y`` of shape (na, nv, nu); returns (nz, ny, nx)."""
    y = np.asarray(y, dtype=np.float64).reshape(g.proj_shape)
    X = _centres(g.nx, g.vx, g.ox)[None, None, :]
    Y = _centres(g.ny, g.vy, g.oy)[None, :, None]
    Z = _centres(g.nz, g.vz, g.oz)[:, None, None]
    cu, cv = (g.nu - 1) / 2.0, (g.nv - 1) / 2.0
    vol = g.vx * g.vy * g.vz
    x = np.zeros(g.vol_shape)
    for a, t in enumerate(g.angles):
        cs, sn = np.cos(t), np.sin(t)
        w = g.dso - (X * cs + Y * sn)
        u = g.dsd * (-X * sn + Y * cs) / w
        v = g.dsd * Z / w
        val = _bilinear(y[a], u / g.du + cu, v / g.dv + cv)
        weight = vol / (g.du * g.dv) * (g.dsd / w) ** 2 * np.sqrt(g.dsd ** 2 + u * u + v * v) / g.dsd
        x += weight * val
    return x
