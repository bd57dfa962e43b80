"""GPU projector parity: the HIP forward and back projectors against the FP64
oracle, element by element, on seeded inputs.

Tolerance: the kernels evaluate the ray geometry in FP64 and accumulate in
FP32, so each ray or voxel sum carries ~1e-7 relative rounding per term and
the whole output a relative L2 error of a few 1e-7.  The gate is 1e-6
relative L2 (and 2e-6 of the output's max per element); 16-bit storage adds
its own output rounding (2^-8 BF16, 2^-11 FP16).
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _geoms():
    return {
        "cgls32": synth.geometry("cgls32"),
        # Ragged tiles in every direction, offsets, anisotropic voxels, odd detector.
        "ragged": synth.geometry(dict(nx=37, ny=29, nz=21, vx=0.9, vy=1.1, vz=1.0, nu=77, nv=45, du=1.1, dv=0.9,
                                      dso=400.0, dsd=640.0, n_angles=23, ox=1.3, oy=-2.1, oz=0.7)),
        # Odd detector at angle 0 (cos, sin exactly 1, 0): the central column
        # and row of rays lie exactly in the y = 0 and z = 0 voxel faces, which
        # the half-open voxel convention assigns to the voxel above.  (At pi/2
        # or pi the computed cos/sin are ~1e-16, not 0, and such rays lie
        # within rounding of a face: which voxel they traverse is then decided
        # by rounding on either side, so only exact angles are tested.)
        "face_planes": synth.geometry(dict(nx=16, ny=16, nz=8, vx=1.0, vy=1.0, vz=1.0, nu=33, nv=17, du=0.8,
                                           dv=0.8, dso=200.0, dsd=300.0, angles=np.array([0.0, 1.0]))),
        "medical_crop": synth.crop_geometry("medical256", 64, 128, 45),
        "muct_crop": synth.crop_geometry("muct1500", 64, 48, 32),
        "torso_crop": synth.geometry(dict(nx=48, ny=48, nz=40, vx=0.5, vy=0.5, vz=0.5, nu=96, nv=72, du=0.4,
                                          dv=0.4, dso=1000.0, dsd=1500.0, n_angles=30)),
        # A detector much finer than the voxels' images (about 10 columns per
        # voxel diagonal), as in the request stream's small-volume cases.
        "fine_detector": synth.geometry(dict(nx=20, ny=20, nz=18, vx=0.5, vy=0.5, vz=0.5, nu=160, nv=150, du=0.1,
                                             dv=0.1, dso=1000.0, dsd=1500.0, n_angles=12)),
    }


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def kct(gpu_lib):
    return gpu_lib


@pytest.mark.parametrize("name", list(_geoms()))
def test_forward_matches_oracle(kct, name):
    gd = _geoms()[name]
    og, kg = oracle.Geometry.from_dict(gd), kct.Geometry.from_dict(gd)
    x = synth.random_volume(og.vol_shape, 100)
    print(f"[forward] {name} vol={og.vol_shape} proj={og.proj_shape}", flush=True)
    plan = kct.Plan(kg)
    y = plan.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
    ref = oracle.forward(og, x)
    assert _rel(y, ref) <= 1e-6
    assert np.max(np.abs(y - ref)) <= 2e-6 * np.max(np.abs(ref))
    assert np.mean(ref > 0) > 0.2


@pytest.mark.parametrize("name", list(_geoms()))
def test_backward_matches_oracle(kct, name):
    gd = _geoms()[name]
    og, kg = oracle.Geometry.from_dict(gd), kct.Geometry.from_dict(gd)
    y = synth.random_projections(og.proj_shape, 101)
    print(f"[backward] {name}", flush=True)
    plan = kct.Plan(kg)
    x = plan.backproject(torch.from_numpy(y).to(DEV)).cpu().numpy()
    ref = oracle.adjoint(og, y)
    assert _rel(x, ref) <= 1e-6
    assert np.max(np.abs(x - ref)) <= 2e-6 * np.max(np.abs(ref))
    plan.check()  # no footprint beyond the plan's bounds


@pytest.mark.parametrize("name", ["cgls32", "ragged", "medical_crop"])
def test_adjoint_identity_fp32(kct, name):
    gd = _geoms()[name]
    kg = kct.Geometry.from_dict(gd)
    plan = kct.Plan(kg)
    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.randn(kg.vol_shape, generator=g).to(DEV)
    y = torch.randn(kg.proj_shape, generator=g).to(DEV)
    Ax = plan.forward(x)
    ATy = plan.backproject(y)
    lhs = float(torch.dot(Ax.double().ravel(), y.double().ravel()))
    rhs = float(torch.dot(x.double().ravel(), ATy.double().ravel()))
    scale = float(Ax.double().norm() * y.double().norm())
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_bitwise_deterministic(kct):
    gd = _geoms()["ragged"]
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    x = torch.from_numpy(synth.random_volume(plan.geom.vol_shape, 5)).to(DEV)
    y = torch.from_numpy(synth.random_projections(plan.geom.proj_shape, 6)).to(DEV)
    assert torch.equal(plan.forward(x), plan.forward(x))
    assert torch.equal(plan.backproject(y), plan.backproject(y))


@pytest.mark.parametrize("name", ["ragged", "face_planes", "muct_crop"])
def test_forward_gather_depths_agree_bitwise(kct, name, monkeypatch):
    """The forward loop gathering 0, 1 or 2 segments ahead (KCT_FWD_PREFETCH,
    read at plan creation) loads the same voxels and adds the same segments
    in the same order: the projections are bitwise equal, for FP32 and FP16
    storage."""
    gd = _geoms()[name]
    x = torch.from_numpy(synth.random_volume(tuple(gd[k] for k in ("nz", "ny", "nx")), 7)).to(DEV)
    outs = []
    for depth in ("0", "1", "2"):
        monkeypatch.setenv("KCT_FWD_PREFETCH", depth)
        plan = kct.Plan(kct.Geometry.from_dict(gd))
        outs.append((plan.forward(x), plan.forward(x.half())))
        torch.cuda.synchronize()
        plan.close()
    for o in outs[1:]:
        assert torch.equal(outs[0][0], o[0]) and torch.equal(outs[0][1], o[1])


@pytest.mark.parametrize("name,lanes", [("ragged", "16"), ("ragged", "64"), ("face_planes", "32"), ("muct_crop", "16")])
def test_forward_workgroup_shapes_agree_bitwise(kct, name, lanes, monkeypatch):
    """Workgroups of one angle (64 x 4 pixels) and of one wave patch at 4, 8
    or 16 angles (KCT_FWD_WAVE_ANGLES), in angle blocks of 4 to 128
    (KCT_FWD_ANGLE_BLOCK), handed to the XCDs in eighths, half row bands or
    turns of 3 tiles (KCT_FWD_XCD_CHUNK; all read at plan creation), trace
    every ray with
    the same code: the projections are bitwise equal, also for the angles of
    a last, partly filled block (23 angles) and ragged detector edges."""
    gd = _geoms()[name]
    x = torch.from_numpy(synth.random_volume(tuple(gd[k] for k in ("nz", "ny", "nx")), 9)).to(DEV)
    monkeypatch.setenv("KCT_FWD_LANES_U", lanes)
    outs = []
    for wa, ab, xc in (("1", "8", "-1"), ("4", "8", "-1"), ("4", "4", "-1"), ("4", "16", "-1"), ("1", "32", "-1"),
                       ("4", "32", "-1"), ("8", "16", "-1"), ("8", "8", "-1"), ("16", "32", "-1"), ("8", "128", "0"),
                       ("4", "64", "0"), ("8", "16", "3")):
        monkeypatch.setenv("KCT_FWD_WAVE_ANGLES", wa)
        monkeypatch.setenv("KCT_FWD_ANGLE_BLOCK", ab)
        monkeypatch.setenv("KCT_FWD_XCD_CHUNK", xc)
        plan = kct.Plan(kct.Geometry.from_dict(gd))
        outs.append(plan.forward(x))
        torch.cuda.synchronize()
        plan.close()
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


@pytest.mark.parametrize("dt", [torch.float16, torch.bfloat16])
def test_forward_16bit_padding_widths_agree_bitwise(kct, dt, monkeypatch):
    """A 16-bit volume's padded copies in FP32 (the default) or in its own
    type (KCT_FWD_PAD_F32=0) hold the same values: the projections are
    bitwise equal, in FP32 and in 16-bit output storage."""
    gd = _geoms()["ragged"]
    x = torch.from_numpy(synth.random_volume(tuple(gd[k] for k in ("nz", "ny", "nx")), 10)).to(DEV).to(dt)
    outs = []
    for wide in ("1", "0"):
        monkeypatch.setenv("KCT_FWD_PAD_F32", wide)
        plan = kct.Plan(kct.Geometry.from_dict(gd))
        outs.append((plan.forward(x, out_dtype=torch.float32), plan.forward(x)))
        torch.cuda.synchronize()
        plan.close()
    assert outs[0][1].dtype == dt
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_backward_angle_split(kct, monkeypatch):
    """Small volumes split the back projector's angles over chunks of
    workgroups (32^3: 16 chunks) and sum the partial volumes in chunk order:
    the result equals the unsplit one (KCT_BWD_SPLIT=1) to FP32 summation
    order, and the plan counts the partial volumes in its device bytes."""
    gd = _geoms()["cgls32"]
    y = torch.from_numpy(synth.random_projections((len(gd["angles"]), gd["nv"], gd["nu"]), 8)).to(DEV)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    split = plan.backproject(y)
    torch.cuda.synchronize()
    assert plan.device_bytes() >= 16 * 32 ** 3 * 4
    monkeypatch.setenv("KCT_BWD_SPLIT", "1")
    plain = kct.Plan(kct.Geometry.from_dict(gd)).backproject(y)
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(split - plain) / torch.linalg.vector_norm(plain))
    print(f"[split] 16 chunks vs 1: rel diff {d:.2e}", flush=True)
    assert d <= 1e-6 and not torch.equal(split, torch.zeros_like(split))


@pytest.mark.parametrize("dt,tol", [(torch.bfloat16, 6e-3), (torch.float16, 8e-4)])
def test_16bit_storage(kct, dt, tol):
    """16-bit inputs and outputs, FP32 accumulation: error = storage rounding."""
    gd = _geoms()["medical_crop"]
    og, kg = oracle.Geometry.from_dict(gd), kct.Geometry.from_dict(gd)
    plan = kct.Plan(kg)
    x16 = torch.from_numpy(synth.random_volume(og.vol_shape, 8)).to(DEV).to(dt)
    y = plan.forward(x16).float().cpu().numpy()
    ref = oracle.forward(og, x16.float().cpu().numpy())  # same rounded input
    assert _rel(y, ref) <= tol
    p16 = torch.from_numpy(synth.random_projections(og.proj_shape, 9)).to(DEV).to(dt)
    xb = plan.backproject(p16).float().cpu().numpy()
    refb = oracle.adjoint(og, p16.float().cpu().numpy())
    assert _rel(xb, refb) <= tol
    # 16-bit projections into an FP32 volume: only input rounding remains.
    xb32 = plan.backproject(p16, out_dtype=torch.float32).cpu().numpy()
    assert _rel(xb32, refb) <= 1e-6


def test_full_size_medical256_sampled(kct):
    """Full 256^3 / 360 x 512^2 geometry in the benchmark's launch shape.
    Forward: every ray of 3 sampled angles against the oracle.  Back projection
    of data that is zero outside 2 sampled angles: every voxel."""
    gd = synth.geometry("medical256")
    kg = kct.Geometry.from_dict(gd)
    og = oracle.Geometry.from_dict(gd)
    print("[full medical256] phantom + forward", flush=True)
    x = synth.phantom("medical256")
    plan = kct.Plan(kg)
    y = plan.forward(torch.from_numpy(x).to(DEV))
    angs = [0, 97, 271]
    ref = oracle.forward(og.with_angles([og.angles[a] for a in angs]), x)
    got = y[angs].cpu().numpy()
    assert _rel(got, ref) <= 1e-6
    del y
    print("[full medical256] back projection", flush=True)
    sel = [45, 200]
    yz = torch.zeros(kg.proj_shape, device=DEV)
    ys = synth.random_projections((len(sel),) + kg.proj_shape[1:], 12)
    yz[sel] = torch.from_numpy(ys).to(DEV)
    xb = plan.backproject(yz).cpu().numpy()
    refb = oracle.adjoint(og.with_angles([og.angles[a] for a in sel]), ys)
    assert _rel(xb, refb) <= 1e-6
    plan.check()  # no footprint beyond the plan's bounds
