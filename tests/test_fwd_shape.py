"""CPU check of the forward projector's launch-shape choice per geometry.

The plan picks the wave patch from the ray spacing at the rotation axis
(32 x 2 pixels when neighbouring rays are a voxel or more apart, else
16 x 4), widens 16-bit volumes into FP32 padded copies while those fit in
4 GiB, and traces one patch at 4 neighbouring angles per workgroup (8 where
the padded copies stay 16-bit), in work-order blocks of 128 angles when the
plan has at least 256 angles, else of 8.  The
choice is computed on the host, without a device; the environment overrides
are checked too."""
import ctypes

import numpy as np
import pytest

import synth
from paper_2211_14212_amd import _lib


def _shape(gd):
    a = np.ascontiguousarray(np.asarray(gd["angles"], dtype=np.float64))
    g = _lib.KctGeometry(gd["nx"], gd["ny"], gd["nz"], gd["vx"], gd["vy"], gd["vz"], gd["ox"], gd["oy"], gd["oz"],
                         gd["nu"], gd["nv"], gd["du"], gd["dv"], gd["dso"], gd["dsd"], len(a),
                         a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    out = [ctypes.c_int() for _ in range(4)]
    rc = _lib.load().kct_debug_fwd_shape_geom(ctypes.byref(g), *(ctypes.byref(o) for o in out))
    assert rc == 0
    return tuple(o.value for o in out)


@pytest.mark.parametrize("name,expect", [
    # 0.4 mm pixels at magnification 1.5: rays 0.27 mm apart, voxels 0.5 mm.
    ("medical256", (16, 4, 128, 1)),
    # 2 x 514^3 FP32 padded copies (1.09 GB) fit in 4 GiB.
    ("torso512", (16, 4, 128, 1)),
    # 0.1 mm pixels at magnification 5.33: rays 18.75 um apart, voxels
    # 10 um; 2 x 1502^3 FP32 copies (27 GB) would not fit in 4 GiB, so the
    # copies stay 16-bit and a workgroup traces 8 angles.
    ("muct1500", (32, 8, 128, 0)),
    # 1 mm pixels at 1.5: rays 0.67 mm apart, voxels 1 mm.
    ("cgls32", (16, 4, 8, 1)),
])
def test_forward_shape_per_workload(name, expect, monkeypatch):
    for var in ("KCT_FWD_LANES_U", "KCT_FWD_WAVE_ANGLES", "KCT_FWD_ANGLE_BLOCK", "KCT_FWD_PAD_F32"):
        monkeypatch.delenv(var, raising=False)
    assert _shape(synth.geometry(name)) == expect


def test_ray_spacing_threshold():
    """Rays exactly one voxel apart at the axis take the wide patch."""
    gd = dict(synth.geometry("cgls32"))
    gd["du"] = gd["vx"] * gd["dsd"] / gd["dso"]  # 1.5 mm pixels: 1 mm at the axis
    assert _shape(gd)[0] == 32
    gd["du"] *= 0.99
    assert _shape(gd)[0] == 16


def test_environment_overrides(monkeypatch):
    gd = synth.geometry("medical256")
    monkeypatch.setenv("KCT_FWD_LANES_U", "64")
    monkeypatch.setenv("KCT_FWD_WAVE_ANGLES", "1")
    monkeypatch.setenv("KCT_FWD_ANGLE_BLOCK", "32")
    monkeypatch.setenv("KCT_FWD_PAD_F32", "0")
    assert _shape(gd) == (64, 1, 32, 0)
    # Values outside the allowed sets are ignored.
    monkeypatch.setenv("KCT_FWD_LANES_U", "48")
    monkeypatch.setenv("KCT_FWD_WAVE_ANGLES", "2")
    monkeypatch.setenv("KCT_FWD_ANGLE_BLOCK", "12")
    assert _shape(gd)[:3] == (16, 4, 128)
    # A block holds at least one workgroup's angles.
    monkeypatch.setenv("KCT_FWD_WAVE_ANGLES", "16")
    monkeypatch.setenv("KCT_FWD_ANGLE_BLOCK", "8")
    assert _shape(gd)[1:3] == (16, 16)
