"""SIRT and OS-SART, the algebraic methods the paper compares with (Sec. 3),
on the GPU against the FP64 oracle.

They are stationary iterations on the FP32 matched projectors, so their
rounding is not amplified the way a Krylov recurrence's is; the gate is 4x
the oracle's own sensitivity to FP32-level matvec noise, never tighter than
1e-5.  OS-SART's subsets are the interleaved angle sets a = k mod m.
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
    b, _ = synth.add_noise(oracle.forward(og, xt), synth.WORKLOADS["cgls32"]["noise"], 1)
    return gpu_lib, gd, og, xt, b.astype(np.float32)


def _perturbed(f, rng):
    def g(z):
        y = f(z)
        return (y * (1 + 5e-7 * rng.standard_normal(y.shape))).astype(np.float32).astype(np.float64)
    return g


def _subsets(og, b, m):
    angs = np.asarray(og.angles)
    subs, bs = [], []
    for k in range(m):
        gk = og.with_angles(angs[k::m])
        subs.append(((lambda v, gk=gk: oracle.forward(gk, v)), (lambda y, gk=gk: oracle.adjoint(gk, y))))
        bs.append(b[k::m])
    return subs, bs


@pytest.mark.parametrize("m", [1, 4])
def test_sart_matches_oracle(problem, m):
    kct, gd, og, xt, b = problem
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    n = 20 if m == 1 else 6
    solver = "sirt" if m == 1 else "os_sart"
    kw = {} if m == 1 else {"n_subsets": m}
    x, h = plan.solve(torch.from_numpy(b).to(DEV), solver, n, 1.0, **kw)
    torch.cuda.synchronize()
    x, h = x.cpu().numpy(), h.cpu().numpy()
    b64 = b.astype(np.float64)
    rng = np.random.default_rng(0)
    if m == 1:
        A, AT = (lambda v: oracle.forward(og, v)), (lambda y: oracle.adjoint(og, y))
        ref, rh = S.sirt(A, AT, b64, n)
        alt, _ = S.sirt(_perturbed(A, rng), _perturbed(AT, rng), b64, n)
    else:
        subs, bs = _subsets(og, b64, m)
        ref, rh = S.os_sart(subs, bs, n)
        alt, _ = S.os_sart([(_perturbed(A, rng), _perturbed(AT, rng)) for A, AT in subs], bs, n)
    sens = _rel(alt, ref)
    err = _rel(x, ref)
    print(f"[{solver} m={m}] n={n}: err {err:.2e} (sensitivity {sens:.2e}); error vs phantom "
          f"{_rel(x.ravel(), xt.ravel()):.4f}", flush=True)
    assert err <= max(1e-5, 4 * sens)
    np.testing.assert_allclose(h[:, 0], rh["res"], rtol=max(1e-5, 4 * sens))
    assert np.all(h[:, 4] == 1.0) and np.all(h[:, 3] == 0)


def test_os_sart_one_subset_is_sirt_and_krylov_is_faster(problem):
    kct, gd, og, xt, b = problem
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    xs, hs = plan.solve(bt, "sirt", 10, 1.0)
    xo, ho = plan.solve(bt, "os_sart", 10, 1.0, n_subsets=1)
    xc, _ = plan.solve(bt, "cgls", 10)
    torch.cuda.synchronize()
    assert torch.equal(xs, xo) and torch.equal(hs, ho)
    # The comparison the paper draws (Sec. 3): after the same number of
    # iterations (one A and one A^T each) the Krylov iterate is much closer.
    e_sirt = _rel(xs.cpu().numpy().ravel(), xt.ravel())
    e_cgls = _rel(xc.cpu().numpy().ravel(), xt.ravel())
    print(f"[sirt vs cgls] 10 iterations: error vs phantom SIRT {e_sirt:.4f}, CGLS {e_cgls:.4f}", flush=True)
    assert e_cgls < e_sirt


def test_sart_parameters_validated(problem):
    kct, gd, og, xt, b = problem
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    bt = torch.from_numpy(b).to(DEV)
    for kw in (dict(solver="sirt", lam=0.0), dict(solver="sirt", lam=2.5), dict(solver="os_sart", lam=1.0),
               dict(solver="os_sart", lam=1.0, n_subsets=37), dict(solver="cgls", lam=0.0, n_subsets=2)):
        solver, lam = kw.pop("solver"), kw.pop("lam")
        with pytest.raises(kct._lib.KctError):
            plan.solve(bt, solver, 3, lam, **kw)
