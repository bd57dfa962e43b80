"""The explicit-residual stop rule (Sec. 3.1.1 and 3.1.2) on the GPU.

With the flag set, CGLS, LSQR and LSMR compute ||b - A x_k|| from the
iterate after every iteration (history column 0) and stop, returning
x_{k-1}, the first time it grows.  Checked here:
  * before the rule fires, the iterates are those of the run without the
    flag (bitwise), and column 0 holds the explicit residual of the oracle's
    own iterates to 1e-4 relative;
  * on a small well-conditioned consistent problem the FP32 recurrences reach
    their rounding floor within a few dozen iterations, where the explicit
    residual starts to fluctuate: the rule fires (code 3 from that row on),
    the returned x is bitwise the iterate of a run stopped one iteration
    before, and the oracle's rule applied to the recorded residuals agrees.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import solvers as S

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def kct(gpu_lib):
    return gpu_lib


@pytest.mark.parametrize("solver", ["cgls", "lsqr", "lsmr"])
def test_rule_quiet_run_matches_plain_run_and_oracle_residuals(kct, solver):
    gd = synth.geometry("cgls32")
    og = oracle.Geometry.from_dict(gd)
    b, _ = synth.add_noise(oracle.forward(og, synth.phantom("cgls32")), synth.WORKLOADS["cgls32"]["noise"], 1)
    b = b.astype(np.float32)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    n = 8
    x0, h0 = plan.solve(bt, solver, n)
    x1, h1 = plan.solve(bt, solver, n, stop_on_residual_increase=True)
    torch.cuda.synchronize()
    h0, h1 = h0.cpu().numpy(), h1.cpu().numpy()
    print(f"[stop rule {solver}] explicit {h1[:, 0]}", flush=True)
    assert np.all(h1[:, 3] == 0), "the rule fired on a short noisy run"
    assert torch.equal(x0, x1)
    np.testing.assert_array_equal(h0[:, 1:3], h1[:, 1:3])
    A, AT = (lambda v: oracle.forward(og, v)), (lambda y: oracle.adjoint(og, y))
    run = getattr(S, solver)
    b64 = b.astype(np.float64)
    its = [run(A, AT, b64, k)[0] for k in range(1, n + 1)]
    k, _, res = S.explicit_residual_stop(A, b64, its)
    assert k is None
    np.testing.assert_allclose(h1[:, 0], res, rtol=1e-4)


@pytest.mark.parametrize("solver", ["cgls", "lsqr"])
def test_rule_fires_at_the_rounding_floor(kct, solver):
    gd = synth.geometry(dict(nx=8, ny=8, nz=2, vx=1.0, vy=1.0, vz=1.0, nu=16, nv=4, du=1.0, dv=1.0, dso=40.0,
                             dsd=60.0, n_angles=12))
    og = oracle.Geometry.from_dict(gd)
    b = oracle.forward(og, synth.random_volume(og.vol_shape, 3)).astype(np.float32)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    n = 200
    x, h = plan.solve(bt, solver, n, stop_on_residual_increase=True)
    torch.cuda.synchronize()
    h = h.cpu().numpy()
    fired = np.flatnonzero(h[:, 3] == 3)
    assert fired.size > 0, "no increase of the explicit residual in 200 FP32 iterations"
    r = int(fired[0])
    print(f"[stop rule {solver}] fired at row {r}: {h[r - 1, 0]:.3e} -> {h[r, 0]:.3e}", flush=True)
    assert r >= 1 and np.all(h[r:, 3] == 3) and np.all(h[:r, 3] == 0)
    k, _, _ = S.explicit_residual_stop(lambda v: v, np.zeros(1), [np.array([v]) for v in h[: r + 1, 0]])
    assert k == r
    xr, _ = plan.solve(bt, solver, r)
    torch.cuda.synchronize()
    assert torch.equal(x, xr)


def test_rule_rejected_where_it_does_not_apply(kct):
    gd = synth.geometry("cgls32")
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.zeros(plan.geom.proj_shape, device=DEV)
    for solver, lam, kw in (("hybrid_lsqr", 1.0, {}), ("ab_gmres", 0.0, {}), ("sirt", 1.0, {}),
                            ("irn_tv_cgls", 1.0, dict(tv_outer=1, tv_inner=1))):
        with pytest.raises(kct._lib.KctError):
            plan.solve(bt, solver, 3, lam, stop_on_residual_increase=True, **kw)
    lib = kct._lib.load()
    for flags, reserved in ((8, 0), (1, 7)):
        p = kct._lib.KctSolveParams(kct._lib.KCT_CGLS, 3, 0.0, 0, 0, 1e-3, 0, 0, 0.0, 0, 0, flags, reserved)
        n = ctypes.c_size_t()
        assert lib.kct_solve_workspace_bytes(plan.handle, ctypes.byref(p), ctypes.byref(n)) != 0


@pytest.mark.parametrize("solver", ["cgls", "lsqr"])
def test_explicit_residual_flag_records_without_stopping(kct, solver):
    """KCT_FLAG_EXPLICIT_RESIDUAL alone: column 0 holds ||b - A x_k|| (checked
    with the plain forward projector after 6 iterations, far above the FP32
    floor where two correct evaluations differ by their own rounding), the
    iterates are those of the run without the flag, and a long run goes on
    through the increases that stop the rule on this problem."""
    gd = synth.geometry(dict(nx=8, ny=8, nz=2, vx=1.0, vy=1.0, vz=1.0, nu=16, nv=4, du=1.0, dv=1.0, dso=40.0,
                             dsd=60.0, n_angles=12))
    og = oracle.Geometry.from_dict(gd)
    b = oracle.forward(og, synth.random_volume(og.vol_shape, 3)).astype(np.float32)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    n = 120
    x0, _ = plan.solve(bt, solver, n)
    x1, h1 = plan.solve(bt, solver, n, explicit_residual=True)
    x6, h6 = plan.solve(bt, solver, 6, explicit_residual=True)
    r = torch.linalg.vector_norm((plan.forward(x6) - bt).double())
    torch.cuda.synchronize()
    h1, h6 = h1.cpu().numpy(), h6.cpu().numpy()
    assert torch.equal(x0, x1)
    assert np.all(h1[:, 3] == 0)
    assert np.any(np.diff(h1[:, 0]) > 0)
    print(f"[explicit {solver}] 6 iterations: recorded {h6[-1, 0]:.6e}, recomputed {float(r):.6e}", flush=True)
    assert h6[-1, 0] > 1e-3 * float(torch.linalg.vector_norm(bt.double()))
    np.testing.assert_allclose(h6[-1, 0], float(r), rtol=1e-5)
