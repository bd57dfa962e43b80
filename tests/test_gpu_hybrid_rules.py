"""Hybrid LSQR with lambda_k chosen at every iteration (Sec. 2.2.2: GCV and
the discrepancy principle) on the GPU against the FP64 oracle.

The device computes the SVD of B_k by one-sided Jacobi and searches lambda_k
with the same grid, golden-section and bisection steps as the oracle.  B_k
itself comes from FP32 matvecs, so lambda_k inherits their rounding: the gate
is 4x the oracle's own sensitivity (every matvec output perturbed by 5e-7
relative noise and rounded to FP32), and never tighter than 1e-5 for x and
1e-6 for lambda_k.
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


@pytest.fixture(scope="module")
def problem(gpu_lib):
    gd = synth.geometry("cgls32")
    og = oracle.Geometry.from_dict(gd)
    xt = synth.phantom("cgls32")
    bc = oracle.forward(og, xt)
    b, _ = synth.add_noise(bc, synth.WORKLOADS["cgls32"]["noise"], 1)
    b = b.astype(np.float32).astype(np.float64)
    nl = float(np.linalg.norm(b - bc) / np.linalg.norm(b))
    return gpu_lib, og, gpu_lib.Geometry.from_dict(gd), b, nl


def _perturbed(f, rng):
    def g(z):
        y = f(z)
        return (y * (1 + 5e-7 * rng.standard_normal(y.shape))).astype(np.float32).astype(np.float64)
    return g


@pytest.mark.parametrize("rule", ["gcv", "dp"])
def test_hybrid_lambda_rule_matches_oracle(problem, rule):
    kct, og, kg, b, nl = problem
    k = 20
    plan = kct.Plan(kg)
    bt = torch.from_numpy(b.astype(np.float32)).to(DEV)
    x, h = plan.solve(bt, "hybrid_lsqr", k, 0.0, lam_rule=rule, noise_level=nl)
    torch.cuda.synchronize()
    x, h = x.cpu().numpy(), h.cpu().numpy()
    A, AT = (lambda v: oracle.forward(og, v)), (lambda y: oracle.adjoint(og, y))
    ref, rh = S.hybrid_lsqr(A, AT, b, k, 0.0, rule=rule, noise_level=nl)
    rng = np.random.default_rng(0)
    alt, ah = S.hybrid_lsqr(_perturbed(A, rng), _perturbed(AT, rng), b, k, 0.0, rule=rule, noise_level=nl)
    sens_x = _rel(alt, ref)
    pos = (rh["lam"] > 0) & (ah["lam"] > 0)
    sens_l = float(np.max(np.abs(ah["lam"][pos] / rh["lam"][pos] - 1))) if pos.any() else 0.0
    lam_gpu = h[:, 4]
    print(f"[hybrid {rule}] nl={nl:.4f} lam_k oracle {rh['lam'][[0, k // 2, k - 1]]} gpu {lam_gpu[[0, k // 2, k - 1]]}; "
          f"x err {_rel(x, ref):.2e} (sens {sens_x:.2e}), lam sens {sens_l:.2e}", flush=True)
    assert _rel(x, ref) <= max(1e-5, 4 * sens_x)
    both = (rh["lam"] > 0) & (lam_gpu > 0)
    # Zero (DP: target not reached yet) on both sides, except possibly at the
    # one iteration where the residual crosses the target.
    assert np.count_nonzero((rh["lam"] > 0) != (lam_gpu > 0)) <= 1
    np.testing.assert_allclose(lam_gpu[both], rh["lam"][both], rtol=max(1e-6, 4 * sens_l))
    np.testing.assert_allclose(h[:, 0], rh["res"], rtol=max(1e-6, 4 * sens_l))
    if rule == "dp":
        assert both.any() and not both.all()
    else:
        assert both.all()


def test_hybrid_rules_validated(problem):
    kct, og, kg, b, nl = problem
    plan = kct.Plan(kg)
    bt = torch.from_numpy(b.astype(np.float32)).to(DEV)
    with pytest.raises(kct._lib.KctError):
        plan.solve(bt, "lsqr", 5, 0.0, lam_rule="gcv")
    with pytest.raises(kct._lib.KctError):
        plan.solve(bt, "hybrid_lsqr", 5, 0.0, lam_rule="dp", noise_level=0.0)
