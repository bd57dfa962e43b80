"""The allocation-free forward projection (kct_forward_noalloc) against
kct_forward, through the C ABI: bitwise the same projections on two calls in a
row on one GPU, the second with a smaller volume (so the second call reads the
static scratch after a larger one left it), for FP32 and FP16 storage; and a
volume whose padded copies exceed the static scratch is refused with
KCT_E_BUDGET before anything is enqueued."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _geom(n, det, na):
    return synth.geometry(dict(nx=n, ny=n + 3, nz=n - 5, vx=0.5, vy=0.5, vz=0.5, nu=det, nv=det - 6, du=0.6, dv=0.6,
                               dso=1000.0, dsd=1500.0, n_angles=na))


@pytest.mark.parametrize("dt", [torch.float32, torch.float16])
def test_forward_noalloc_matches_forward(gpu_lib, dt):
    kct = gpu_lib
    for n, det, na, seed in ((160, 200, 24, 81), (48, 72, 10, 82)):
        print(f"[noalloc] {n} voxels, {det} pixels, {na} angles, {dt}", flush=True)
        plan = kct.Plan(kct.Geometry.from_dict(_geom(n, det, na)))
        x = torch.from_numpy(synth.random_volume(plan.geom.vol_shape, seed)).to(DEV).to(dt)
        ref = plan.forward(x)
        out = torch.full(plan.geom.proj_shape, float("nan"), device=DEV, dtype=dt)
        plan.forward_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, dt)
        plan.close()


def test_forward_noalloc_refuses_beyond_its_scratch(gpu_lib):
    kct = gpu_lib
    plan = kct.Plan(kct.Geometry.from_dict(_geom(300, 64, 2)))  # 2 x 302 x 305 x 297 FP32 > 128 MiB
    x = torch.zeros(plan.geom.vol_shape, device=DEV)
    out = torch.full(plan.geom.proj_shape, 7.0, device=DEV)
    with pytest.raises(kct._lib.KctError) as e:
        plan.forward_noalloc(x, out)
    assert "KCT_E_BUDGET" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)  # nothing was enqueued
    plan.close()
