"""Every launch shape of the matched back projector against the FP64 oracle,
element by element, with data on every angle.

The plan picks the back projector's shape from the geometry: voxels per
thread along z (KZ = 16, 8 or 1), where the per-voxel sums live (LDS or
registers), the angle split of small volumes, and, when every voxel's
footprint is narrower than one detector pixel in both directions (the
micro-CT magnification), the ray-driven tile kernel.  The environment
overrides read at plan creation force each shape on the same inputs, so
every code path is compared with the oracle's scatter adjoint, not only the
one the default choice takes.

Gate as for the other projector tests: relative L2 <= 1e-6 and every element
within 2e-6 of the output's maximum (FP64 geometry, FP32 sums).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def kct(gpu_lib):
    return gpu_lib


def _geoms():
    return {
        "medical_crop": synth.crop_geometry("medical256", 64, 128, 45),
        "muct_crop": synth.crop_geometry("muct1500", 64, 48, 32),
        # A 192^3 request-sized volume (0.5 mm voxels, 384^2 detector whose
        # field of view is 1.1x the volume): its default shape is KZ = 8.
        "mid192": synth.geometry(dict(nx=192, ny=192, nz=192, vx=0.5, vy=0.5, vz=0.5, nu=384, nv=384,
                                      du=1.1 * 192 * 0.5 * 1.5 / 384, dv=1.1 * 192 * 0.5 * 1.5 / 384,
                                      dso=1000.0, dsd=1500.0, n_angles=6)),
    }


def _check(kct, gd, seed):
    og, kg = oracle.Geometry.from_dict(gd), kct.Geometry.from_dict(gd)
    y = synth.random_projections(og.proj_shape, seed)
    plan = kct.Plan(kg)
    shape = plan.bwd_shape()
    x = plan.backproject(torch.from_numpy(y).to(DEV)).cpu().numpy()
    plan.check()  # no footprint beyond the plan's bounds
    ref = oracle.adjoint(og, y)
    rel = _rel(x, ref)
    print(f"    shape {shape}: rel L2 {rel:.2e}", flush=True)
    assert np.count_nonzero(ref) > 0.5 * ref.size
    assert rel <= 1e-6
    assert np.max(np.abs(x - ref)) <= 2e-6 * np.max(np.abs(ref))
    return shape


# (geometry, forced KZ, forced accumulator place, forced angle split, forced kernel)
SHAPES = [
    ("medical_crop", "1", None, None, None),
    ("medical_crop", "8", "1", None, None),
    ("medical_crop", "8", "0", None, None),
    ("medical_crop", "16", "1", None, None),
    ("medical_crop", "16", "0", None, None),
    ("medical_crop", "16", "1", "1", None),
    ("muct_crop", "8", "1", None, "0"),
    ("muct_crop", "16", "1", None, "0"),
    ("muct_crop", "16", "1", "1", "0"),
    ("muct_crop", None, None, None, None),
    ("muct_crop", None, None, "1", None),
]


@pytest.mark.parametrize("name,kz,acc,split,rays", SHAPES)
def test_backward_shape_matches_oracle(kct, name, kz, acc, split, rays, monkeypatch):
    monkeypatch.delenv("KCT_BWD_XCD_CHUNK", raising=False)
    for var, val in (("KCT_BWD_KZ", kz), ("KCT_BWD_ACC", acc), ("KCT_BWD_SPLIT", split), ("KCT_BWD_RAYS", rays)):
        if val is not None:
            monkeypatch.setenv(var, val)
        else:
            monkeypatch.delenv(var, raising=False)
    print(f"[bwd shape] {name} KZ={kz} ACC={acc} SPLIT={split} RAYS={rays}", flush=True)
    shape = _check(kct, _geoms()[name], 211)
    if kz is not None:
        assert shape["kz"] == int(kz)


@pytest.mark.parametrize("name,rays", [("medical_crop", "0"), ("muct_crop", None)])
def test_backward_xcd_turns_agree_bitwise(kct, name, rays, monkeypatch):
    """The order in which the XCDs take the tiles (KCT_BWD_XCD_CHUNK: one
    contiguous eighth each, or turns of 1, 3 or 32 tiles) changes no voxel's
    sum: each tile's sums are formed by one workgroup alone."""
    for var in ("KCT_BWD_KZ", "KCT_BWD_ACC", "KCT_BWD_SPLIT"):
        monkeypatch.delenv(var, raising=False)
    if rays is None:
        monkeypatch.delenv("KCT_BWD_RAYS", raising=False)
    else:
        monkeypatch.setenv("KCT_BWD_RAYS", rays)
    gd = _geoms()[name]
    y = torch.from_numpy(synth.random_projections(tuple(
        (len(gd["angles"]), gd["nv"], gd["nu"])), 214)).to(DEV)
    outs = []
    for c in ("-1", "1", "3", "32"):
        monkeypatch.setenv("KCT_BWD_XCD_CHUNK", c)
        plan = kct.Plan(kct.Geometry.from_dict(gd))
        outs.append(plan.backproject(y))
        torch.cuda.synchronize()
        plan.close()
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


def test_backward_default_shape_mid_volume(kct, monkeypatch):
    """A 192^3 volume takes KZ = 8 by default (too few 16-deep tiles to fill
    the GPU several times over) and no angle split."""
    for var in ("KCT_BWD_KZ", "KCT_BWD_ACC", "KCT_BWD_SPLIT", "KCT_BWD_RAYS"):
        monkeypatch.delenv(var, raising=False)
    print("[bwd shape] mid192 default", flush=True)
    shape = _check(kct, _geoms()["mid192"], 212)
    assert shape["kz"] == 8 and shape["split"] == 1 and shape["rays"] == 0


def test_ray_backprojector_bitwise_deterministic(kct, monkeypatch):
    """The ray-driven kernel adds every voxel's terms in a fixed order (angle
    order within each of its four copies of the tile sums, then the copies in
    order): two runs give the same bits, with and without the angle split."""
    for var in ("KCT_BWD_KZ", "KCT_BWD_ACC", "KCT_BWD_RAYS"):
        monkeypatch.delenv(var, raising=False)
    gd = _geoms()["muct_crop"]
    y = torch.from_numpy(synth.random_projections(tuple(
        (len(gd["angles"]), gd["nv"], gd["nu"])), 213)).to(DEV)
    for split in ("1", "16"):
        monkeypatch.setenv("KCT_BWD_SPLIT", split)
        plan = kct.Plan(kct.Geometry.from_dict(gd))
        assert plan.bwd_shape()["rays"] == 1
        a, b = plan.backproject(y), plan.backproject(y)
        torch.cuda.synchronize()
        assert torch.equal(a, b), split
        plan.close()
