"""CPU check that the back projector's launch-shape bounds hold.

The kernel stages, per angle, the detector patch of a 16 x 16 x KZ voxel
tile in LDS and unrolls a fixed number of candidate columns per voxel.  The
host derives both sizes from a magnification bound; here they are checked
against the footprints computed exactly (FP64 perspective projection of the
corners) for every tile and angle of reduced-size workloads and sampled
tiles of the full-size ones."""
import ctypes
import math

import numpy as np
import pytest

import synth
from paper_2211_14212_amd import _lib


def _shape(gd):
    a = np.ascontiguousarray(np.asarray(gd["angles"], dtype=np.float64))
    g = _lib.KctGeometry(gd["nx"], gd["ny"], gd["nz"], gd["vx"], gd["vy"], gd["vz"], gd["ox"], gd["oy"], gd["oz"],
                         gd["nu"], gd["nv"], gd["du"], gd["dv"], gd["dso"], gd["dsd"], len(a),
                         a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    kz, nc, pw, ph = (ctypes.c_int() for _ in range(4))
    rc = _lib.load().kct_debug_bwd_shape_geom(ctypes.byref(g), ctypes.byref(kz), ctypes.byref(nc),
                                             ctypes.byref(pw), ctypes.byref(ph))
    assert rc == 0
    return kz.value, nc.value, pw.value, ph.value


def _footprints(gd, x0, x1, y0, y1, z0, z1, angles):
    """Exact pixel-index extents (float) of boxes [x0,x1]x[y0,y1]x[z0,z1] (arrays)."""
    cs, sn = np.cos(angles)[:, None], np.sin(angles)[:, None]
    us, ws = [], []
    for x in (x0, x1):
        for y in (y0, y1):
            w = gd["dso"] - (x[None] * cs + y[None] * sn)
            us.append(gd["dsd"] * (-x[None] * sn + y[None] * cs) / w)
            ws.append(w)
    u = np.stack(us)
    w = np.stack(ws)
    vs = [gd["dsd"] * z[None] / ww for z in (z0, z1) for ww in (w.min(0), w.max(0))]
    v = np.stack(vs)
    ucols = u.max(0) / gd["du"] - u.min(0) / gd["du"]
    vrows = v.max(0) / gd["dv"] - v.min(0) / gd["dv"]
    return ucols, vrows


@pytest.mark.parametrize("name,crop", [("cgls32", None), ("medical256", None), ("torso512", None),
                                       ("muct1500", None), ("serve_big", None), ("serve_fine", None)])
def test_launch_bounds_are_conservative(name, crop):
    if name == "serve_big":
        gd = synth.geometry(dict(nx=512, ny=512, nz=512, vx=0.5, vy=0.5, vz=0.5, nu=256, nv=256,
                                 du=1.1 * 512 * 0.5 * 1.5 / 256, dv=1.1 * 512 * 0.5 * 1.5 / 256, dso=1000.0,
                                 dsd=1500.0, n_angles=90))
    elif name == "serve_fine":
        # The request stream's finest case: 128^3 on a 1024^2 detector, about
        # 7 pixels per voxel width.
        gd = synth.geometry(dict(nx=128, ny=128, nz=128, vx=0.5, vy=0.5, vz=0.5, nu=1024, nv=1024,
                                 du=1.1 * 128 * 0.5 * 1.5 / 1024, dv=1.1 * 128 * 0.5 * 1.5 / 1024, dso=1000.0,
                                 dsd=1500.0, n_angles=90))
    else:
        gd = synth.geometry(name)
    kz, ncm, pw, ph = _shape(gd)
    rng = np.random.default_rng(0)
    angles = np.asarray(gd["angles"])
    angles = angles[rng.choice(angles.size, min(angles.size, 64), replace=False)]
    X0 = gd["ox"] - gd["nx"] * gd["vx"] / 2
    Y0 = gd["oy"] - gd["ny"] * gd["vy"] / 2
    Z0 = gd["oz"] - gd["nz"] * gd["vz"] / 2
    # Every voxel column (sampled for big grids): per-voxel column count.
    n_col = min(gd["nx"] * gd["ny"], 4096)
    ci = rng.integers(0, gd["nx"], n_col)
    cj = rng.integers(0, gd["ny"], n_col)
    x0 = X0 + ci * gd["vx"]
    y0 = Y0 + cj * gd["vy"]
    ucols, _ = _footprints(gd, x0, x0 + gd["vx"], y0, y0 + gd["vy"], np.zeros(n_col), np.zeros(n_col), angles)
    # Integers inside an interval of this length (plus the kernel's 0.01-pixel margins).
    max_cols = int(math.floor(ucols.max() + 0.02)) + 1
    assert max_cols <= ncm, (max_cols, ncm)
    # Tiles: 16 x 16 x kz voxels.
    tx = np.arange(0, gd["nx"], 16)
    ty = np.arange(0, gd["ny"], 16)
    tzs = np.arange(0, gd["nz"], kz)
    T = np.array([(a, b, c) for a in tx for b in ty for c in tzs])
    if len(T) > 4096:
        T = T[rng.choice(len(T), 4096, replace=False)]
    ie = np.minimum(T[:, 0] + 16, gd["nx"])
    je = np.minimum(T[:, 1] + 16, gd["ny"])
    ke = np.minimum(T[:, 2] + kz, gd["nz"])
    uc, vr = _footprints(gd, X0 + T[:, 0] * gd["vx"], X0 + ie * gd["vx"], Y0 + T[:, 1] * gd["vy"],
                         Y0 + je * gd["vy"], Z0 + T[:, 2] * gd["vz"], Z0 + ke * gd["vz"], angles)
    assert int(math.floor(uc.max() + 0.02)) + 1 <= pw
    assert int(math.floor(vr.max() + 0.02)) + 1 <= ph
