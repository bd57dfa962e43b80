"""Solver parity against the FP64 oracle at the full 256^3 benchmark size.

Workload: the 256^3 ellipsoid phantom at 0.5 mm, 360 angles of a 512^2
detector at 0.4 mm (DSO 1000 mm, DSD 1500 mm), Poisson counts at I0 = 1e5:
the configuration the benchmark times, in the launch shapes it uses.  The
projections b are the oracle's own forward projection of the phantom with
the seeded Poisson noise, rounded to FP32; both sides read the same b.

Three iterations of each solver (each oracle product takes about 16 s on 16
host threads).  CGLS and LSQR produce the same iterates in exact arithmetic
(Sec. 2.1.2; pinned on the CPU to 1e-10), so both GPU runs are compared with
the oracle's CGLS; LSMR with the oracle's LSMR.  Gate: relative L2 <= 1e-5.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import solvers as S

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
K = 3


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def medical(gpu_lib):
    kct = gpu_lib
    gd = synth.geometry("medical256")
    og = oracle.Geometry.from_dict(gd)
    t0 = time.perf_counter()
    xt = synth.phantom("medical256")
    b, _ = synth.add_noise(oracle.forward(og, xt), synth.WORKLOADS["medical256"]["noise"],
                           synth.WORKLOADS["medical256"]["seed"])
    print(f"[full oracle] medical256 b from the oracle ({time.perf_counter() - t0:.0f} s)", flush=True)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    yield og, plan, b
    plan.close()


def _ops(og):
    def A(v):
        t0 = time.perf_counter()
        y = oracle.forward(og, v)
        print(f"    oracle A ({time.perf_counter() - t0:.0f} s)", flush=True)
        return y

    def AT(y):
        t0 = time.perf_counter()
        x = oracle.adjoint(og, y)
        print(f"    oracle A^T ({time.perf_counter() - t0:.0f} s)", flush=True)
        return x

    return A, AT


def test_cgls_and_lsqr_full_size(medical):
    og, plan, b = medical
    bt = torch.from_numpy(b).to(DEV)
    xc, hc = plan.solve(bt, "cgls", K)
    xl, hl = plan.solve(bt, "lsqr", K)
    torch.cuda.synchronize()
    print(f"[full oracle] CGLS-{K}", flush=True)
    ref, rh = S.cgls(*_ops(og), b.astype(np.float64), K)
    ec, el = _rel(xc.cpu().numpy(), ref), _rel(xl.cpu().numpy(), ref)
    print(f"[full oracle] GPU CGLS-{K} {ec:.2e}, GPU LSQR-{K} {el:.2e} vs oracle CGLS-{K}", flush=True)
    assert ec <= 1e-5 and el <= 1e-5
    np.testing.assert_allclose(hc.cpu().numpy()[:, 0], rh["res"], rtol=1e-5)
    np.testing.assert_allclose(hl.cpu().numpy()[:, 0], rh["res"], rtol=1e-5)


def test_lsmr_full_size(medical):
    og, plan, b = medical
    bt = torch.from_numpy(b).to(DEV)
    x, h = plan.solve(bt, "lsmr", K)
    torch.cuda.synchronize()
    print(f"[full oracle] LSMR-{K}", flush=True)
    ref, rh = S.lsmr(*_ops(og), b.astype(np.float64), K)
    e = _rel(x.cpu().numpy(), ref)
    print(f"[full oracle] GPU LSMR-{K} {e:.2e} vs oracle LSMR-{K}", flush=True)
    assert e <= 1e-5
    np.testing.assert_allclose(h.cpu().numpy()[:, 0], rh["normal"], rtol=1e-5)
