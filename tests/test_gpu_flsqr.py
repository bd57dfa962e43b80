"""Hybrid fLSQR-TV (Sec. 2.3.2) on the GPU against the FP64 oracle.

The oracle and the device take the same steps: x0 from the best constant,
the flexible Golub-Kahan process with full modified Gram-Schmidt on both
bases, (L D)^+ applied by the same number of CG steps, and the projected
Tikhonov solve with lambda_k fixed or by GCV.  The gate is 4x the oracle's own
sensitivity to FP32-level noise on every matvec output, never tighter than
2e-5.  With eps = 0.1 the weights are smooth functions of the iterate and the
run is well conditioned (the sensitivity stays below 1e-6 at 8 iterations).
With eps = 1e-3 the weights of nearly flat regions swing with rounding-level
changes of the iterate: the sensitivity is 2e-4 at 4 iterations and 5e-3 at
8.  The inner CG on the weighted Laplacian, badly conditioned there, runs in
FP64 on the device; in FP32 it alone moved the 4-iteration result by 1.1e-3
(oracle runs with FP32 CG vectors), five times the matvec effect.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import solvers as S

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _perturbed(f, rng):
    def g(z):
        y = f(z)
        return (y * (1 + 5e-7 * rng.standard_normal(y.shape))).astype(np.float32).astype(np.float64)
    return g


@pytest.fixture(scope="module")
def problem(gpu_lib):
    gd = synth.geometry("cgls32")
    og = oracle.Geometry.from_dict(gd)
    xt = synth.phantom("cgls32")
    b, _ = synth.add_noise(oracle.forward(og, xt), synth.WORKLOADS["cgls32"]["noise"], 1)
    return gpu_lib, gd, og, xt, b.astype(np.float32)


@pytest.mark.parametrize("rule,lam,eps,n", [("fixed", 1.0, 0.1, 8), ("fixed", 10.0, 0.1, 8), ("gcv", 0.0, 0.1, 8),
                                            ("fixed", 3.0, 1e-3, 4), ("fixed", 3.0, 1e-3, 8)])
def test_flsqr_tv_matches_oracle(problem, rule, lam, eps, n):
    kct, gd, og, xt, b = problem
    J = 10
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    x, h = plan.solve(torch.from_numpy(b).to(DEV), "hybrid_flsqr_tv", n, lam, lam_rule=rule, tv_inner=J, tv_eps=eps)
    torch.cuda.synchronize()
    x, h = x.cpu().numpy(), h.cpu().numpy()
    A, AT = (lambda v: oracle.forward(og, v)), (lambda y: oracle.adjoint(og, y))
    b64 = b.astype(np.float64)
    ref, rh = S.hybrid_flsqr_tv(A, AT, b64, og.vol_shape, n, lam, eps, J, rule=rule)
    rng = np.random.default_rng(0)
    alt, _ = S.hybrid_flsqr_tv(_perturbed(A, rng), _perturbed(AT, rng), b64, og.vol_shape, n, lam, eps, J, rule=rule)
    sens = _rel(alt, ref)
    err = _rel(x, ref)
    gate = max(2e-5, 4 * sens)
    print(f"[flsqr-tv {rule} lam={lam} eps={eps} n={n}] err {err:.2e} (sensitivity {sens:.2e}); lam_k {h[-1, 4]:.4g} vs "
          f"{rh['lam'][-1]:.4g}; error vs phantom {_rel(x.ravel(), xt.ravel()):.4f}", flush=True)
    assert err <= gate
    np.testing.assert_allclose(h[:, 0], rh["res"], rtol=gate)
    np.testing.assert_allclose(h[:, 4], rh["lam"], rtol=gate if rule == "gcv" else 0)
    M = rh["M"]
    np.testing.assert_allclose(h[:, 2], [M[k + 1, k] for k in range(n)], rtol=max(1e-4, 40 * sens))
    assert np.all(h[:, 3] == 0)


def test_flsqr_tv_constant_image_and_zero_iterations(problem):
    kct, gd, og, xt, b = problem
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bc = oracle.forward(og, np.full(og.vol_shape, 0.7)).astype(np.float32)
    x, h = plan.solve(torch.from_numpy(bc).to(DEV), "hybrid_flsqr_tv", 3, 1.0, tv_inner=5, tv_eps=1e-3)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    print(f"[flsqr-tv constant] max |x - 0.7| = {np.abs(x - 0.7).max():.2e}", flush=True)
    np.testing.assert_allclose(x, 0.7, rtol=2e-5)
    # Zero iterations leave x0, the best constant fit of b.
    x0, _ = plan.solve(torch.from_numpy(b).to(DEV), "hybrid_flsqr_tv", 0, 1.0, tv_inner=5, tv_eps=1e-3)
    torch.cuda.synchronize()
    _, rh = S.hybrid_flsqr_tv(lambda v: oracle.forward(og, v), lambda y: oracle.adjoint(og, y),
                              b.astype(np.float64), og.vol_shape, 0, 1.0, 1e-3, 5)
    np.testing.assert_allclose(x0.cpu().numpy(), rh["x0"], rtol=1e-5)


def test_flsqr_tv_parameters_validated(problem):
    kct, gd, og, xt, b = problem
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    for kw in (dict(tv_inner=0), dict(tv_inner=5, tv_outer=2), dict(tv_inner=5, tv_eps=0.0),
               dict(tv_inner=5, vec_dtype=torch.bfloat16)):
        with pytest.raises(kct._lib.KctError):
            plan.solve(bt, "hybrid_flsqr_tv", 3, 1.0, **kw)


def test_flsqr_tv_full_size_residual_identity(gpu_lib):
    """At the benchmark's 256^3 / 360 x 512^2 size: with orthonormal u_i the
    projected residual equals the explicit ||A x_k - b|| (lambda ~ 0), which
    checks the flexible relation A Z_k = U_{k+1} M_k and x = x0 + Z_k y at
    full size with the GPU's own matched forward projector."""
    kct = gpu_lib
    gd = synth.geometry("medical256")
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    xt = torch.from_numpy(synth.phantom("medical256")).to(DEV)
    b = plan.forward(xt)
    b, _ = synth.add_noise_torch(b, synth.WORKLOADS["medical256"]["noise"], 2)
    x, h = plan.solve(b, "hybrid_flsqr_tv", 6, 1e-6, tv_inner=5, tv_eps=0.1)
    r = plan.forward(x) - b
    torch.cuda.synchronize()
    explicit = float(torch.linalg.vector_norm(r.double()))
    h = h.cpu().numpy()
    print(f"[flsqr-tv medical256] projected {h[-1, 0]:.6e} explicit {explicit:.6e}; residuals {h[:, 0]}", flush=True)
    assert np.all(np.diff(h[:, 0]) <= 0)
    assert abs(h[-1, 0] - explicit) <= 2e-4 * explicit
