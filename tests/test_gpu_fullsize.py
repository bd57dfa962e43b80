"""Full-size parity for the two large workloads, in the launch configuration
the benchmark uses (whole geometry, every angle), checked on outputs the FP64
oracle can compute at modest cost.

- 512^3 torso shape (1024 x 768 detector, 720 angles): every ray of three
  sampled angles of the forward projection, and the back projection of data
  that is zero outside one angle, against the oracle on the full geometry.
- 1500^3 micro-CT shape (2000^2 detector, 1571 angles): the volume is zero
  outside two voxel blocks.  A Siddon line integral only sums the voxels a ray
  crosses, so each ray's value equals the sum, over the blocks, of the same
  ray's integral through a volume that is just that block (same source,
  detector and voxel grid).  The oracle evaluates those block geometries; the
  GPU runs the full 1500^3 problem.  The back projection of data that is zero
  outside two angles is compared on the block voxels the same way.

Tolerances as in the small parity tests: FP64 geometry with FP32
accumulation gives a relative L2 error of a few 1e-7; the gate is 1e-6.  FP16
projection storage adds its output rounding (2^-11 relative).
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


def test_full_size_torso512_sampled(kct):
    gd = synth.geometry("torso512")
    kg, og = kct.Geometry.from_dict(gd), oracle.Geometry.from_dict(gd)
    print("[full torso512] random volume + forward (720 angles)", flush=True)
    x = synth.random_volume(og.vol_shape, 31)
    plan = kct.Plan(kg)
    y = plan.forward(torch.from_numpy(x).to(DEV))
    angs = [0, 250, 611]
    got = y[angs].cpu().numpy()
    del y
    ref = oracle.forward(og.with_angles([og.angles[a] for a in angs]), x)
    assert _rel(got, ref) <= 1e-6
    print("[full torso512] back projection of one angle", flush=True)
    sel = [377]
    ys = synth.random_projections((1,) + kg.proj_shape[1:], 32)
    yz = torch.zeros(kg.proj_shape, device=DEV)
    yz[sel] = torch.from_numpy(ys).to(DEV)
    xb = plan.backproject(yz).cpu().numpy()
    del yz
    refb = oracle.adjoint(og.with_angles([og.angles[a] for a in sel]), ys)
    assert _rel(xb, refb) <= 1e-6
    plan.check()  # no footprint beyond the plan's bounds


def test_full_size_muct1500_blocks(kct):
    gd = synth.geometry("muct1500")
    kg = kct.Geometry.from_dict(gd)
    blocks = [((726, 726, 726), (48, 48, 48)), ((100, 1290, 402), (32, 40, 36))]
    vals = [synth.random_volume(s, 41 + n) for n, (_, s) in enumerate(blocks)]
    bgs = [oracle.Geometry.from_dict(synth.block_geometry(gd, o, s)) for (o, s) in blocks]
    print("[full muct1500] block-supported volume + forward (1571 angles)", flush=True)
    x = torch.zeros(kg.vol_shape, device=DEV)
    for (o, s), v in zip(blocks, vals):
        x[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]] = torch.from_numpy(v).to(DEV)
    plan = kct.Plan(kg)
    angs = [0, 393, 1100]
    ref = sum(oracle.forward(bg.with_angles([gd["angles"][a] for a in angs]), v) for bg, v in zip(bgs, vals))
    y = plan.forward(x)
    got = y[angs].cpu().numpy()
    del y
    assert np.count_nonzero(ref) > 1000
    assert _rel(got, ref) <= 1e-6
    print("[full muct1500] FP16 projection storage", flush=True)
    y16 = plan.forward(x, out_dtype=torch.float16)
    got16 = y16[angs].float().cpu().numpy()
    del y16
    assert _rel(got16, ref) <= 1e-3
    del x
    print("[full muct1500] back projection of two angles", flush=True)
    sel = [71, 980]
    ys = synth.random_projections((len(sel),) + kg.proj_shape[1:], 43)
    yz = torch.zeros(kg.proj_shape, device=DEV)
    yz[sel] = torch.from_numpy(ys).to(DEV)
    xb = plan.backproject(yz)
    del yz
    for (o, s), bg in zip(blocks, bgs):
        gotb = xb[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]].cpu().numpy()
        refb = oracle.adjoint(bg.with_angles([gd["angles"][a] for a in sel]), ys)
        assert np.count_nonzero(refb) > 100
        assert _rel(gotb, refb) <= 1e-6
    plan.check()  # no footprint beyond the plan's bounds


def test_full_size_solver_identities(kct):
    """Solver parity at the benchmark's and the torso's full sizes, through
    identities that hold at any size (the oracle would need minutes per
    product here):
    - 256^3 / 360 x 512^2 (the benchmark's launch configuration): CGLS and
      LSQR produce the same iterates in exact arithmetic (Sec. 2.1.2), and
      CGLS's recurred residual equals the explicit ||b - A x_k||;
    - 512^3 / 720 x 1024 x 768: hybrid LSQR with a fixed lambda equals damped
      LSQR (Sec. 2.2.1) iterate by iterate.
    Gates: 1e-5 relative (the FP32 rounding of 10 iterations)."""
    gd = synth.geometry("medical256")
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    print("[full medical256] phantom, projections, CGLS-10 and LSQR-10", flush=True)
    xt = torch.from_numpy(synth.phantom("medical256")).to(DEV)
    b, _ = synth.add_noise_torch(plan.forward(xt), synth.WORKLOADS["medical256"]["noise"], 2)
    xc, hc = plan.solve(b, "cgls", 10)
    xl, hl = plan.solve(b, "lsqr", 10)
    r = torch.linalg.vector_norm((plan.forward(xc) - b).double())
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(xc - xl) / torch.linalg.vector_norm(xc))
    print(f"[full medical256] CGLS vs LSQR {d:.2e}; recurred {float(hc[-1, 0]):.6e} explicit {float(r):.6e}",
          flush=True)
    assert d <= 1e-5
    assert abs(float(hc[-1, 0]) - float(r)) <= 1e-5 * float(r)
    np.testing.assert_allclose(hc[:, 0].cpu().numpy(), hl[:, 0].cpu().numpy(), rtol=1e-5)
    del xt, b, xc, xl, plan
    torch.cuda.empty_cache()

    gd = synth.geometry("torso512")
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    print("[full torso512] random volume, projections, LSQR-10 and hybrid LSQR-10 at lambda 10", flush=True)
    x = torch.from_numpy(synth.random_volume(plan.geom.vol_shape, 33)).to(DEV)
    b = plan.forward(x)
    del x
    xd, hd = plan.solve(b, "lsqr", 10, 10.0)
    xh, hh = plan.solve(b, "hybrid_lsqr", 10, 10.0)
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(xd - xh) / torch.linalg.vector_norm(xd))
    print(f"[full torso512] damped LSQR vs hybrid {d:.2e}", flush=True)
    assert d <= 1e-5
