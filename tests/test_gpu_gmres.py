"""The unmatched interpolating back projector B and AB-/BA-GMRES (Sec. 2.1.4)
on the GPU against the FP64 oracle.

B: FP64 projection of voxel centres, FP32 bilinear weights and sums; gate
1e-6 relative L2 as for the matched projectors.  GMRES: with B = A^T the
iterates are LSQR's (AB) and LSMR's (BA), checked against the library's own
LSQR and LSMR; with the interpolating B they are checked against the
oracle's GMRES on the oracle's B, gated at 4x the oracle's sensitivity to
FP32-level matvec noise (never tighter than 1e-5).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import solvers as S
from oracle.interp import backproject_interp

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def kct(gpu_lib):
    return gpu_lib


GEOMS = {
    "cgls32": lambda: synth.geometry("cgls32"),
    "ragged": lambda: synth.geometry(dict(nx=37, ny=29, nz=21, vx=0.9, vy=1.1, vz=1.0, nu=77, nv=45, du=1.1,
                                          dv=0.9, dso=400.0, dsd=640.0, n_angles=23, ox=1.3, oy=-2.1, oz=0.7)),
    "medical_crop": lambda: synth.crop_geometry("medical256", 64, 128, 45),
}


@pytest.mark.parametrize("name", list(GEOMS))
def test_interp_backprojector_matches_oracle(kct, name):
    gd = GEOMS[name]()
    og, kg = oracle.Geometry.from_dict(gd), kct.Geometry.from_dict(gd)
    y = synth.random_projections(og.proj_shape, 7)
    plan = kct.Plan(kg)
    got = plan.backproject_interp(torch.from_numpy(y).to(DEV)).cpu().numpy()
    ref = backproject_interp(og, y)
    print(f"[interp B] {name}: rel {_rel(got, ref):.2e}", flush=True)
    assert _rel(got, ref) <= 1e-6


def _cgls32():
    gd = synth.geometry("cgls32")
    og = oracle.Geometry.from_dict(gd)
    xt = synth.phantom("cgls32")
    b, _ = synth.add_noise(oracle.forward(og, xt), synth.WORKLOADS["cgls32"]["noise"], 1)
    return gd, og, b.astype(np.float32)


def test_gmres_with_matched_backprojector_is_lsqr_and_lsmr(kct):
    gd, og, b = _cgls32()
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    k = 15
    xa, ha = plan.solve(bt, "ab_gmres", k)
    xq, hq = plan.solve(bt, "lsqr", k)
    xb, hb = plan.solve(bt, "ba_gmres", k)
    xm, _ = plan.solve(bt, "lsmr", k)
    torch.cuda.synchronize()
    assert _rel(xa.cpu().numpy(), xq.cpu().numpy()) <= 1e-5
    assert _rel(xb.cpu().numpy(), xm.cpu().numpy()) <= 1e-5
    # AB-GMRES's residual is LSQR's ||b - A x_k|| (undamped).
    np.testing.assert_allclose(ha.cpu().numpy()[:, 0], hq.cpu().numpy()[:, 0], rtol=1e-4)
    assert np.all(np.diff(hb.cpu().numpy()[:, 0]) <= 0)


def _perturbed(f, rng):
    def g(z):
        y = f(z)
        return (y * (1 + 5e-7 * rng.standard_normal(y.shape))).astype(np.float32).astype(np.float64)
    return g


@pytest.mark.parametrize("solver", ["ab_gmres", "ba_gmres"])
def test_gmres_with_interp_backprojector_matches_oracle(kct, solver):
    gd, og, b = _cgls32()
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    k = 12
    x, h = plan.solve(torch.from_numpy(b).to(DEV), solver, k, backprojector="interp")
    torch.cuda.synchronize()
    x, h = x.cpu().numpy(), h.cpu().numpy()
    A = lambda v: oracle.forward(og, v)
    B = lambda y: backproject_interp(og, y)
    fn = getattr(S, solver)
    ref, rh = fn(A, B, b.astype(np.float64), k)
    rng = np.random.default_rng(0)
    alt, _ = fn(_perturbed(A, rng), _perturbed(B, rng), b.astype(np.float64), k)
    sens = _rel(alt, ref)
    err = _rel(x, ref)
    print(f"[{solver} interp] k={k}: err {err:.2e}, sensitivity {sens:.2e}; res {h[-1, 0]:.6g} vs {rh['res'][-1]:.6g}",
          flush=True)
    assert err <= max(1e-5, 4 * sens)
    np.testing.assert_allclose(h[:, 0], rh["res"], rtol=max(1e-5, 4 * sens))


def test_gmres_parameters_validated(kct):
    gd, og, b = _cgls32()
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    with pytest.raises(kct._lib.KctError):
        plan.solve(bt, "lsqr", 3, backprojector="interp")
    with pytest.raises(kct._lib.KctError):
        plan.solve(bt, "ab_gmres", 3, lam=1.0)
    with pytest.raises(kct._lib.KctError):
        plan.solve(bt, "ba_gmres", 3, vec_dtype=torch.float16)
