"""Pins of the oracle's hybrid fLSQR-TV (Sec. 2.3.2, eq. (TV_standard_form))
to things other than itself:

  * the pieces of the standard-form transform against dense linear algebra:
    the inner CG against numpy's pseudoinverse of L D, the closed-form
    projector E against the paper's definition of the A-weighted
    pseudoinverse [I - (A (I - (LD)^+ L D))^+ A] (LD)^+, and x0 against the
    least-squares fit of b by A on the null space (the constants);
  * with L held at I and exact inner solves, n - 1 iterations reach the
    dense solution of the general-form Tikhonov problem
    min ||A x - b||^2 + lam^2 ||D x||^2;
  * the flexible relations A Z = U M with orthonormal U and V, and the
    projected solution equal to the direct minimiser of
    ||A (x0 + Z y) - b||^2 + lam^2 ||y||^2 over y;
  * a constant image is recovered from its own projections.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense
from oracle import solvers as S


def _problem(seed=0, noise=0.01):
    g = oracle.Geometry(nx=4, ny=3, nz=2, vx=1.0, vy=1.0, vz=1.0, nu=8, nv=5, du=1.0, dv=1.0,
                        dso=20.0, dsd=32.0, angles=tuple(synth.angles(8, start=0.3)))
    A = dense.system_matrix(g)
    shape = g.vol_shape
    xt = synth.random_volume(shape, seed).astype(np.float64)
    b = A @ xt.ravel() + noise * np.random.default_rng(seed).standard_normal(A.shape[0])
    return A, b, shape


def _ops(A, shape):
    return (lambda x: A @ x.ravel()), (lambda y: (A.T @ y).reshape(shape))


def _dense_D(shape):
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(S.grad(e.reshape(shape)).ravel())
    return np.stack(cols, axis=1)  # (3n, n)


def test_pseudoinverse_pieces_against_dense():
    A, b, shape = _problem()
    n = int(np.prod(shape))
    rng = np.random.default_rng(1)
    Lw = 0.3 + rng.random(shape)
    LD = np.tile(Lw.ravel(), 3)[:, None] * _dense_D(shape)
    LDp = np.linalg.pinv(LD)
    # (L D)^+ v = K^+ D^T L v by CG.
    v = rng.standard_normal(3 * n)
    t = S.cg_weighted_laplacian(Lw * Lw, S.grad_T(Lw[None] * v.reshape((3,) + shape)), 200)
    np.testing.assert_allclose(t.ravel(), LDp @ v, rtol=0, atol=1e-10 * np.linalg.norm(LDp @ v))
    # ((L D)^+)^T w = L D K^+ w for w orthogonal to the constants.
    w = rng.standard_normal(n)
    w -= w.mean()
    u = Lw[None] * S.grad(S.cg_weighted_laplacian(Lw * Lw, w.reshape(shape), 200))
    np.testing.assert_allclose(u.ravel(), LDp.T @ w, rtol=0, atol=1e-10 * np.linalg.norm(LDp.T @ w))
    # A-weighted pseudoinverse: the paper's definition vs E (L D)^+.
    # (A N)^+ with N the rank-1 projector I - (LD)^+ L D; the cutoff drops the
    # rounding-level singular values of the dense product.
    LA = (np.eye(n) - np.linalg.pinv(A @ (np.eye(n) - LDp @ LD), rcond=1e-8) @ A) @ LDp
    a = A @ np.ones(n)
    g = A.T @ a
    E = np.eye(n) - np.outer(np.ones(n), g) / (a @ a)
    np.testing.assert_allclose(E @ LDp, LA, rtol=0, atol=1e-10 * np.abs(LA).max())
    # x0: the constant that best fits b.
    Aop, ATop = _ops(A, shape)
    _, h = S.hybrid_flsqr_tv(Aop, ATop, b, shape, 1, 1.0, 1e-3, 50)
    c = np.linalg.lstsq(a[:, None], b, rcond=None)[0][0]
    np.testing.assert_allclose(h["x0"], np.full(shape, c), rtol=1e-13)


@pytest.mark.parametrize("lam", [0.3, 3.0])
def test_fixed_weights_reach_general_form_tikhonov(lam):
    A, b, shape = _problem(seed=2)
    n = int(np.prod(shape))
    D = _dense_D(shape)
    ref = np.linalg.solve(A.T @ A + lam * lam * (D.T @ D), A.T @ b)
    Aop, ATop = _ops(A, shape)
    x, h = S.hybrid_flsqr_tv(Aop, ATop, b, shape, n - 1, lam, 1e-3, 300, reweight=False)
    assert len(h["Z"]) == n - 1
    np.testing.assert_allclose(x.ravel(), ref, rtol=0, atol=1e-9 * np.linalg.norm(ref))
    # The last projected residual is that of the general-form problem.
    bbar = b - A @ h["x0"].ravel()
    full = np.sqrt(np.sum((A @ ref - b) ** 2) + lam * lam * np.sum((D @ ref) ** 2))
    assert abs(h["res"][-1] - full) <= 1e-9 * np.linalg.norm(bbar)


@pytest.mark.parametrize("rule", ["fixed", "gcv"])
def test_flexible_relations_and_projected_solution(rule):
    A, b, shape = _problem(seed=3)
    Aop, ATop = _ops(A, shape)
    k, lam = 8, 0.5
    x, h = S.hybrid_flsqr_tv(Aop, ATop, b, shape, k, lam, 1e-2, 30, rule=rule)
    U = np.stack([u.ravel() for u in h["U"]], axis=1)
    V = np.stack([v.ravel() for v in h["V"]], axis=1)
    Z = np.stack([z.ravel() for z in h["Z"]], axis=1)
    M = h["M"]
    assert U.shape[1] == k + 1 and V.shape[1] == k and M.shape == (k + 1, k)
    np.testing.assert_allclose(U.T @ U, np.eye(k + 1), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(A @ Z, U @ M, atol=1e-12 * np.abs(A @ Z).max())
    assert np.all(np.tril(M, -2) == 0.0)
    # Direct minimiser over x0 + span(Z) with the same lam_k.
    lk = h["lam"][-1]
    r0 = b - A @ h["x0"].ravel()
    K = np.vstack([A @ Z, lk * np.eye(k)])
    y = np.linalg.lstsq(K, np.concatenate([r0, np.zeros(k)]), rcond=None)[0]
    np.testing.assert_allclose(x.ravel(), h["x0"].ravel() + Z @ y, rtol=0, atol=1e-10 * np.linalg.norm(x))
    assert abs(h["res"][-1] - np.linalg.norm(K @ y - np.concatenate([r0, np.zeros(k)]))) <= 1e-10 * np.linalg.norm(r0)
    # The weights change between iterations: the basis is really flexible.
    xf, _ = S.hybrid_flsqr_tv(Aop, ATop, b, shape, k, lam, 1e-2, 30, rule=rule, reweight=False)
    assert np.linalg.norm(xf - x) > 1e-3 * np.linalg.norm(x)


def test_constant_image_is_recovered():
    A, _, shape = _problem()
    Aop, ATop = _ops(A, shape)
    b = A @ np.full(int(np.prod(shape)), 0.7)
    x, h = S.hybrid_flsqr_tv(Aop, ATop, b, shape, 3, 1.0, 1e-3, 20)
    np.testing.assert_allclose(x, 0.7, rtol=1e-9)
