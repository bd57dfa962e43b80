"""Pins of the oracle's unmatched back projector B (Sec. 2.1.4), CPU only.

Hand-derived cases: a 5^3 grid of unit voxels centred on the axis (centres at
-2..2 mm), DSO = 100, DSD = 200, angle 0 (source on +x, detector plane
x = -100, e_u = +y, e_v = +z).  A voxel centre (0, y, z) projects to
u = 2y, v = 2z, i.e. magnification 2.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.interp import backproject_interp

GD = dict(nx=5, ny=5, nz=5, vx=1.0, vy=1.0, vz=1.0, nu=9, nv=9, du=2.0, dv=2.0, dso=100.0, dsd=200.0,
          angles=(0.0,))


def _g(**kw):
    d = dict(GD)
    d.update(kw)
    return oracle.Geometry.from_dict(d)


def test_voxel_on_pixel_centre():
    """du = 2: the voxel centre (0, y, z) lands on pixel (iu, iv) = (y + 4,
    z + 4), so B y there is weight * y[iv, iu] with weight =
    V/(du dv) (DSD/w)^2 |d|/DSD = 1/4 * 4 * sqrt(200^2 + (2y)^2 + (2z)^2)/200."""
    g = _g()
    y = np.zeros((1, 9, 9))
    y[0, 4 + 1, 4 - 2] = 3.0   # the pixel under voxel centre (0, -2, 1)
    x = backproject_interp(g, y)
    k, j, i = 1 + 2, -2 + 2, 0 + 2
    expect = 3.0 * math.sqrt(200.0 ** 2 + 4.0 ** 2 + 2.0 ** 2) / 200.0
    assert x[k, j, i] == pytest.approx(expect, rel=1e-14)
    # Every other voxel of that x = 0 slice lands on a zero pixel.
    sl = x[:, :, i].copy()
    sl[k, j] = 0.0
    assert np.all(sl == 0.0)


def test_half_pixel_interpolates_midpoint():
    """du = 4: the centre (0, 1, 0) lands half-way between pixel columns 4 and
    5 of row 4, so it receives the mean of the two values times the weight
    1/8 * 4 * sqrt(200^2 + 2^2)/200 (dv stays 2)."""
    g = _g(du=4.0)
    y = np.zeros((1, 9, 9))
    y[0, 4, 4], y[0, 4, 5] = 1.0, 5.0
    x = backproject_interp(g, y)
    w = 1.0 / 8.0 * 4.0 * math.sqrt(200.0 ** 2 + 2.0 ** 2) / 200.0
    assert x[2, 3, 2] == pytest.approx(w * 3.0, rel=1e-14)


def test_off_detector_is_zero():
    """A 3-pixel detector only sees the centre: every voxel whose image falls
    outside the pixel grid gets zero, whatever the data."""
    g = _g(nu=3, nv=3, du=1.0, dv=1.0)
    x = backproject_interp(g, np.ones((1, 3, 3)))
    # Images at u = 2y, v = 2z (x = 0 slice): inside only for |2y|, |2z| <= 1.
    assert x[2, 2, 2] > 0
    assert x[2, 0, 2] == 0.0 and x[0, 2, 2] == 0.0 and x[4, 4, 2] == 0.0


def test_close_to_exact_transpose_on_smooth_data():
    """On constant data B 1 approximates A^T 1 (the total ray length through
    each voxel): pixels several times finer than the voxels' images, many
    angles.  The weight's (DSD/w)^2 |d|/DSD factor is what makes the two agree
    across the volume; the Siddon adjoint is the oracle pinned elsewhere."""
    d = dict(nx=12, ny=12, nz=8, vx=1.0, vy=1.0, vz=1.0, nu=96, nv=64, du=0.35, dv=0.35, dso=60.0, dsd=120.0,
             angles=tuple(np.linspace(0, 2 * np.pi, 24, endpoint=False)))
    g = oracle.Geometry.from_dict(d)
    ones = np.ones(g.proj_shape)
    ratio = backproject_interp(g, ones) / oracle.adjoint(g, ones)
    inner = ratio[1:-1, 1:-1, 1:-1]
    assert abs(inner.mean() - 1.0) < 0.02
    assert np.all(np.abs(inner - 1.0) < 0.15)
