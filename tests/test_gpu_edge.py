"""Degenerate shapes on the GPU: single voxels, single pixels, a single
angle, a one-slice volume, rays that miss the volume, and solvers asked for
zero iterations.  Projector results against the FP64 oracle, same gate as
the other projector tests (1e-6 relative L2)."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _rel(a, b):
    n = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / n) if n > 0 else float(np.linalg.norm(a))


@pytest.fixture(scope="module")
def kct(gpu_lib):
    return gpu_lib


EDGE = {
    "one_voxel": dict(nx=1, ny=1, nz=1, vx=1.0, vy=1.0, vz=1.0, nu=5, nv=5, du=0.7, dv=0.7, dso=10.0, dsd=20.0,
                      n_angles=7),
    "one_pixel": dict(nx=4, ny=5, nz=3, vx=1.0, vy=1.0, vz=1.0, nu=1, nv=1, du=1.0, dv=1.0, dso=30.0, dsd=50.0,
                      n_angles=9),
    "one_angle": dict(nx=9, ny=7, nz=5, vx=1.0, vy=1.2, vz=0.8, nu=16, nv=12, du=1.1, dv=0.9, dso=60.0, dsd=90.0,
                      n_angles=1),
    "one_slice": dict(nx=24, ny=24, nz=1, vx=1.0, vy=1.0, vz=1.0, nu=40, nv=3, du=1.0, dv=0.6, dso=80.0,
                      dsd=120.0, n_angles=8),
    # Offset volume: most rays of the detector miss it.
    "mostly_missing": dict(nx=6, ny=6, nz=6, vx=1.0, vy=1.0, vz=1.0, nu=70, nv=70, du=1.0, dv=1.0, dso=50.0,
                           dsd=80.0, n_angles=5, ox=9.0, oy=-7.0, oz=3.0),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_projectors_on_degenerate_shapes(kct, name):
    gd = synth.geometry(dict(EDGE[name]))
    og, kg = oracle.Geometry.from_dict(gd), kct.Geometry.from_dict(gd)
    plan = kct.Plan(kg)
    x = synth.random_volume(og.vol_shape, 3)
    y = synth.random_projections(og.proj_shape, 4)
    gf = plan.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
    gb = plan.backproject(torch.from_numpy(y).to(DEV)).cpu().numpy()
    rf, rb = oracle.forward(og, x), oracle.adjoint(og, y)
    print(f"[edge] {name}: fwd {_rel(gf, rf):.2e} bwd {_rel(gb, rb):.2e}, nonzero rays {np.count_nonzero(rf)}",
          flush=True)
    assert np.count_nonzero(rf) > 0
    assert _rel(gf, rf) <= 1e-6 and _rel(gb, rb) <= 1e-6
    plan.check()  # no footprint beyond the plan's bounds


@pytest.mark.parametrize("solver,kw", [("cgls", {}), ("lsqr", {}), ("lsmr", {}), ("hybrid_lsqr", {}),
                                       ("hybrid_lsqr", {"lam_rule": "gcv"}), ("ab_gmres", {}), ("ba_gmres", {}),
                                       ("sirt", {"lam": 1.0}), ("os_sart", {"lam": 1.0, "n_subsets": 3})])
def test_zero_iterations_give_zero(kct, solver, kw):
    gd = synth.geometry(dict(EDGE["one_angle"], n_angles=6))
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    b = torch.from_numpy(synth.random_projections(plan.geom.proj_shape, 5)).to(DEV)
    x = torch.full(plan.geom.vol_shape, 7.0, device=DEV)
    kw = dict(kw)
    lam = kw.pop("lam", 0.0)
    x, h = plan.solve(b, solver, 0, lam, x=x, **kw)
    torch.cuda.synchronize()
    assert torch.count_nonzero(x) == 0


def test_irn_tv_single_inner_step(kct):
    gd = synth.geometry(dict(EDGE["one_slice"]))
    og, kg = oracle.Geometry.from_dict(gd), kct.Geometry.from_dict(gd)
    from oracle import solvers as S

    b = oracle.forward(og, synth.random_volume(og.vol_shape, 8)).astype(np.float32)
    plan = kct.Plan(kg)
    x, h = plan.solve(torch.from_numpy(b).to(DEV), "irn_tv_cgls", 0, 0.5, tv_outer=1, tv_inner=1, tv_eps=1e-3)
    torch.cuda.synchronize()
    ref, _ = S.irn_tv_cgls(lambda v: oracle.forward(og, v), lambda y: oracle.adjoint(og, y), b.astype(np.float64),
                           og.vol_shape, 1, 1, 0.5, 1e-3)
    assert _rel(x.cpu().numpy(), ref) <= 1e-5


def test_footprint_overflow_is_reported(kct, monkeypatch):
    """A back projection whose footprint exceeds the plan's bound never passes
    silently.  The overflow is forced from the host (a patch-width bound of 2
    columns, far below this geometry's 13); every access stays inside the
    smaller patch.  kct_plan_check then fails and a solve records code 4."""
    gd = synth.geometry(dict(nx=24, ny=24, nz=8, vx=1.0, vy=1.0, vz=1.0, nu=48, nv=16, du=1.0, dv=1.0, dso=80.0,
                             dsd=120.0, n_angles=6))
    kg = kct.Geometry.from_dict(gd)
    y = torch.from_numpy(synth.random_projections(kg.proj_shape, 9)).to(DEV)
    clean = kct.Plan(kg)
    clean.backproject(y)
    clean.check()
    _, h = clean.solve(y, "cgls", 3)
    assert torch.count_nonzero(h[:, 3]) == 0
    monkeypatch.setenv("KCT_BWD_TEST_PW_MAX", "2")
    plan = kct.Plan(kg)
    plan.backproject(y)
    with pytest.raises(kct.KctError) as err:
        plan.check()
    assert err.value.name == "KCT_E_GEOMETRY"
    plan.check()  # the flag was cleared by the failing check
    for solver in ("cgls", "lsqr"):
        _, h = plan.solve(y, solver, 3)
        assert torch.all(h[:, 3] == 4.0), (solver, h[:, 3])
    with pytest.raises(kct.KctError):
        plan.check()
