"""IRN-TV and 16-bit vector storage on the GPU, against the FP64 oracle.

IRN-TV: the GPU runs the same outer/inner schedule as the oracle (weights from
the previous outer iterate, L = I at the first; inner CGLS restarted), gate
relative L2 <= 1e-5.

16-bit storage (BF16, FP16) of the vectors the projectors read and write,
with FP32 accumulation and FP64 Krylov scalars.  These bounds are empirical
(no closed form exists): measured on these workloads and set with margin,
relative L2 against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import solvers as S

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)

# Empirical bounds of the 16-bit paths (relative L2 vs the FP64 oracle).
MIXED_BOUND = {torch.bfloat16: 2e-2, torch.float16: 3e-3}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def kct(gpu_lib):
    return gpu_lib


def _muct_crop(n=32, det=40, na=24):
    gd = synth.crop_geometry("muct1500", n, det, na)
    og = oracle.Geometry.from_dict(gd)
    xt = synth.phantom("muct1500", gd, full_n=1500, crop_origin=(734, 734, 734))
    b, _ = synth.add_noise(oracle.forward(og, xt), dict(kind="gaussian", rel_sigma=0.01), 4)
    return gd, og, xt, b.astype(np.float32)


@pytest.mark.parametrize("outer,inner,lam", [(1, 6, 0.05), (3, 8, 0.05), (2, 5, 0.5)])
def test_irn_tv_matches_oracle(kct, outer, inner, lam):
    gd, og, xt, b = _muct_crop()
    print(f"[irn-tv] {outer}x{inner} lam={lam}", flush=True)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    eps = 1e-3
    x, h = plan.solve(torch.from_numpy(b).to(DEV), "irn_tv_cgls", 0, lam, tv_outer=outer, tv_inner=inner,
                      tv_eps=eps)
    torch.cuda.synchronize()
    ref, rh = S.irn_tv_cgls(lambda v: oracle.forward(og, v), lambda y: oracle.adjoint(og, y),
                            b.astype(np.float64), og.vol_shape, outer, inner, lam, eps)
    assert _rel(x.cpu().numpy(), ref) <= 1e-5
    np.testing.assert_allclose(h.cpu().numpy()[:, 0], rh["res"], rtol=1e-5)
    assert float(S.tv(x.cpu().numpy().astype(np.float64))) > 0


# The micro-CT workload's TV setting (lambda 10, eps 1e-3) in its storage: the
# projection-side vectors in FP16, x and the Krylov scalars as always.  A
# shortened schedule (3 outer x 10 inner) on the 32^3 crop.  The FP32 path is
# held to the solver gate; the FP16 bound is empirical (measured on this
# crop, see the DESIGN notes on 16-bit storage), relative L2 against the FP64
# oracle.
IRN_MUCT_BOUND = {torch.float32: 1e-5, torch.float16: 3e-3}


@pytest.mark.parametrize("dt", [torch.float32, torch.float16])
def test_irn_tv_muct_setting(kct, dt):
    gd, og, xt, b = _muct_crop()
    outer, inner, lam, eps = 3, 10, 10.0, 1e-3
    print(f"[irn-tv muct] {outer}x{inner} lam={lam} {dt}", flush=True)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    x, h = plan.solve(torch.from_numpy(b).to(DEV), "irn_tv_cgls", 0, lam, vec_dtype=dt, tv_outer=outer,
                      tv_inner=inner, tv_eps=eps)
    torch.cuda.synchronize()
    ref, _ = S.irn_tv_cgls(lambda v: oracle.forward(og, v), lambda y: oracle.adjoint(og, y),
                           b.astype(np.float64), og.vol_shape, outer, inner, lam, eps)
    e = _rel(x.cpu().numpy(), ref)
    print(f"[irn-tv muct] {dt}: rel L2 vs FP64 oracle {e:.2e}", flush=True)
    assert torch.all(torch.isfinite(x)) and torch.all(h[:, 3] == 0)
    assert e <= IRN_MUCT_BOUND[dt]


def test_irn_tv_outer_restart_reduces_tv(kct):
    """More outer reweighting steps lower the TV of the reconstruction relative
    to the same number of plain CGLS steps with the L = I penalty."""
    gd, og, xt, b = _muct_crop()
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    x1, _ = plan.solve(bt, "irn_tv_cgls", 0, 0.5, tv_outer=1, tv_inner=20, tv_eps=1e-3)
    x4, _ = plan.solve(bt, "irn_tv_cgls", 0, 0.5, tv_outer=4, tv_inner=20, tv_eps=1e-3)
    torch.cuda.synchronize()
    assert S.tv(x4.cpu().numpy().astype(np.float64)) < S.tv(x1.cpu().numpy().astype(np.float64))


def _medical_crop():
    gd = synth.crop_geometry("medical256", 48, 96, 40)
    og = oracle.Geometry.from_dict(gd)
    xt = synth.ellipsoid_phantom(gd, 12, (1.0, 6.0), (0.1, 1.0), 2)
    b, _ = synth.add_noise(oracle.forward(og, xt), dict(kind="poisson", i0=1e5), 2)
    return gd, og, b.astype(np.float32)


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("solver,lam", [("lsqr", 0.0), ("cgls", 0.0), ("lsmr", 0.0), ("lsqr", 10.0)])
def test_16bit_vectors_bounded(kct, dt, solver, lam):
    gd, og, b = _medical_crop()
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    x16, h16 = plan.solve(bt, solver, 30, lam, vec_dtype=dt)
    x32, _ = plan.solve(bt, solver, 30, lam)
    torch.cuda.synchronize()
    ref, _ = getattr(S, solver)(lambda v: oracle.forward(og, v), lambda y: oracle.adjoint(og, y),
                                b.astype(np.float64), 30, lam)
    e16 = _rel(x16.cpu().numpy(), ref)
    e32 = _rel(x32.cpu().numpy(), ref)
    print(f"[mixed] {solver} lam={lam} {dt}: rel L2 vs FP64 oracle {e16:.2e} (FP32 path {e32:.2e})", flush=True)
    assert torch.all(torch.isfinite(x16)) and torch.all(h16[:, 3] == 0)
    assert e16 <= MIXED_BOUND[dt]
    assert e32 <= 1e-5
