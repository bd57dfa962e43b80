"""Pins of the oracle's TV operators and IRN-TV loop (Sec. 2.3).

  * D^T is the adjoint of D; D of a linear ramp is its slope (zero at the last
    index, the Neumann reading of the unstated boundary condition);
  * TV (eq. (TV)) of a constant is 0 and of a voxel-aligned step is the face
    area times the jump;
  * the IRN quadratic built from the weights majorises the smoothed TV and
    touches it at the point the weights come from;
  * one outer step with many inner CGLS steps equals the dense solve of
    (A^T A + lam^2 D^T L^2 D) x = A^T b;
  * with converged inner solves the outer iterates decrease the smoothed TV
    objective (the majorise-minimise property of Sec. 2.3).
"""
import numpy as np

import oracle
import synth
from oracle import dense
from oracle import solvers as S


def _dense_grad(shape):
    n = int(np.prod(shape))
    G = np.zeros((3 * n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        G[:, j] = S.grad(e.reshape(shape)).ravel()
    return G


def test_grad_adjoint_and_ramp():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 6, 7))
    g = rng.standard_normal((3, 5, 6, 7))
    assert abs(np.sum(S.grad(x) * g) - np.sum(x * S.grad_T(g))) < 1e-12 * np.abs(x).sum() * np.abs(g).max()
    k, j, i = np.meshgrid(np.arange(5), np.arange(6), np.arange(7), indexing="ij")
    ramp = 0.5 * i - 2.0 * j + 3.0 * k
    d = S.grad(ramp)
    np.testing.assert_allclose(d[0][:, :, :-1], 0.5)
    np.testing.assert_allclose(d[1][:, :-1, :], -2.0)
    np.testing.assert_allclose(d[2][:-1, :, :], 3.0)
    assert np.all(d[0][:, :, -1] == 0) and np.all(d[1][:, -1, :] == 0) and np.all(d[2][-1] == 0)


def test_tv_closed_forms():
    assert S.tv(np.full((4, 5, 6), 3.7)) == 0.0
    x = np.zeros((4, 5, 6))
    x[:, :, 2:] = 1.5  # a jump of 1.5 across one x-face of area 4*5 voxels
    assert abs(S.tv(x) - 1.5 * 4 * 5) < 1e-12
    y = np.zeros((4, 5, 6))
    y[2:, :, :] = -2.0
    assert abs(S.tv(y) - 2.0 * 5 * 6) < 1e-12


def test_irn_majorant_tight():
    rng = np.random.default_rng(1)
    xk = rng.standard_normal((4, 4, 4))
    eps = 1e-2
    lw = S.irn_weights(xk, eps)  # w^{-1/2}
    w = 1.0 / lw ** 2

    def tv_eps(z):
        g = S.grad(z)
        return np.sum(np.sqrt(np.sum(g * g, axis=0) + eps * eps))

    def quad(z):
        g = S.grad(z)
        return 0.5 * np.sum((np.sum(g * g, axis=0) + eps * eps) / w + w)

    assert abs(quad(xk) - tv_eps(xk)) < 1e-12 * tv_eps(xk)
    for s in range(5):
        z = xk + rng.standard_normal(xk.shape)
        assert quad(z) >= tv_eps(z) - 1e-12


def _tiny_tv_problem():
    g = oracle.Geometry(nx=4, ny=4, nz=3, vx=1.0, vy=1.0, vz=1.0, nu=8, nv=5, du=1.0, dv=1.0,
                        dso=20.0, dsd=32.0, angles=tuple(synth.angles(4, start=0.1)))
    A = dense.system_matrix(g)
    shape = g.vol_shape
    xt = np.zeros(shape)
    xt[:, 1:3, 1:3] = 1.0
    b = A @ xt.ravel() + 0.05 * np.random.default_rng(2).standard_normal(A.shape[0])

    def Af(x):
        return A @ x.ravel()

    def ATf(y):
        return (A.T @ y).reshape(shape)

    return A, b, shape, Af, ATf


def test_irn_inner_cgls_matches_dense_solve():
    A, b, shape, Af, ATf = _tiny_tv_problem()
    lam, eps = 0.7, 1e-2
    G = _dense_grad(shape)
    n = A.shape[1]
    # Outer 0: L = I.  (60 inner steps converge: cond < 1e2; far beyond
    # convergence the recurred residual of plain CGLS drifts.)
    x1, _ = S.irn_tv_cgls(Af, ATf, b, shape, 1, 60, lam, eps)
    x1_dense = np.linalg.solve(A.T @ A + lam ** 2 * G.T @ G, A.T @ b)
    np.testing.assert_allclose(x1.ravel(), x1_dense, rtol=0, atol=1e-8 * np.abs(x1_dense).max())
    # Outer 1: weights from x1, restarted CGLS from x1.
    x2, _ = S.irn_tv_cgls(Af, ATf, b, shape, 2, 60, lam, eps)
    lw = np.tile(S.irn_weights(x1_dense.reshape(shape), eps).ravel(), 3)
    x2_dense = np.linalg.solve(A.T @ A + lam ** 2 * G.T @ (lw[:, None] ** 2 * G), A.T @ b)
    np.testing.assert_allclose(x2.ravel(), x2_dense, rtol=0, atol=1e-7 * np.abs(x2_dense).max())
    assert n == G.shape[1]


def test_irn_objective_decreases():
    A, b, shape, Af, ATf = _tiny_tv_problem()
    lam, eps = 0.7, 1e-2

    def objective(x):
        g = S.grad(x)
        return np.sum((A @ x.ravel() - b) ** 2) + lam ** 2 * 2.0 * np.sum(np.sqrt(np.sum(g * g, axis=0) + eps ** 2))

    vals = []
    for n_outer in range(2, 6):
        x, _ = S.irn_tv_cgls(Af, ATf, b, shape, n_outer, 60, lam, eps)
        vals.append(objective(x))
    assert np.all(np.diff(vals) <= 1e-9 * vals[0]), vals
