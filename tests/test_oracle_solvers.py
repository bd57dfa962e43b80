"""Pins of the oracle's FP64 Krylov solvers to things other than themselves.

  * Krylov-subspace optimality, the definition the paper gives for each
    method: CGLS/LSQR minimise ||A x - b|| (Sec. 2.1.1, eq.
    (lest_squares_projected); Sec. 2.1.2, eq. (proj_LSQR)) and LSMR minimises
    ||A^T r|| (Sec. 2.1.3, eq. (proj_LSMR)) over K_k(A^T A, A^T b), checked
    against an explicitly built and twice-orthonormalised Krylov basis;
  * SciPy's independent LSQR and LSMR (damped and undamped), iterate by iterate;
  * dense least squares and damped normal equations at convergence
    (Sec. 2.2, eqs. (Tikhonov) and (Tikhonov_augmented));
  * CGLS == LSQR iterates (Sec. 2.1.2) and hybrid(lambda) == damped LSQR
    (Sec. 2.2.1) in exact arithmetic;
  * monotone residuals (Sec. 2.1.1: ||r_k|| decreases; LSMR: ||A^T r_k||);
  * the recurred norms equal explicitly computed ones;
  * breakdown with b = 0 or A^T b = 0 returns zero without NaN.
"""
import math

import numpy as np
import pytest
from scipy.sparse.linalg import lsmr as scipy_lsmr
from scipy.sparse.linalg import lsqr as scipy_lsqr

import oracle
import synth
from oracle import dense
from oracle import solvers as S


def _ct_problem(seed=0):
    """A tiny cone-beam problem with its dense A (well inside brute-force size)."""
    g = oracle.Geometry(nx=6, ny=6, nz=4, vx=1.0, vy=1.0, vz=1.0, nu=10, nv=6, du=1.0, dv=1.0,
                        dso=20.0, dsd=32.0, angles=tuple(synth.angles(8, start=0.2)))
    A = dense.system_matrix(g)
    xt = synth.random_volume(g.vol_shape, seed).astype(np.float64).ravel()
    b = A @ xt + 0.01 * np.random.default_rng(seed).standard_normal(A.shape[0])
    return A, b


def _random_problem(m=50, n=20, cond=30.0, seed=0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -math.log10(cond), n)
    return (U * s) @ V.T, rng.standard_normal(m)


def _ops(A):
    return (lambda x: A @ x), (lambda y: A.T @ y)


def _krylov_basis(A, b, k):
    K = [A.T @ b]
    for _ in range(k - 1):
        K.append(A.T @ (A @ K[-1]))
    K = np.array(K).T
    K = K / np.linalg.norm(K, axis=0)
    Q, _ = np.linalg.qr(K)
    Q, _ = np.linalg.qr(Q)  # second pass for orthogonality
    return Q


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_krylov_optimality(k):
    A, b = _random_problem(cond=10.0, seed=k)
    Af, ATf = _ops(A)
    V = _krylov_basis(A, b, k)
    y_ls, *_ = np.linalg.lstsq(A @ V, b, rcond=None)
    x_ls = V @ y_ls
    # LSMR: minimise ||A^T (b - A V y)|| = || A^T b - (A^T A V) y ||.
    y_mr, *_ = np.linalg.lstsq(A.T @ (A @ V), A.T @ b, rcond=None)
    x_mr = V @ y_mr
    for fn, want in ((S.cgls, x_ls), (S.lsqr, x_ls), (S.lsmr, x_mr)):
        x, _ = fn(Af, ATf, b, k)
        assert np.linalg.norm(x - want) <= 1e-9 * np.linalg.norm(want), fn.__name__
    # The two criteria really differ at this k (so a swap would be caught).
    if k >= 2:
        assert np.linalg.norm(x_ls - x_mr) > 1e-6 * np.linalg.norm(x_ls)


@pytest.mark.parametrize("lam", [0.0, 0.7])
def test_against_scipy(lam):
    for prob in (_random_problem(cond=50.0, seed=3), _ct_problem(1)):
        A, b = prob
        Af, ATf = _ops(A)
        for k in (1, 3, 6, 8):
            x, _ = S.lsqr(Af, ATf, b, k, lam)
            xs = scipy_lsqr(A, b, damp=lam, atol=0, btol=0, conlim=0, iter_lim=k)[0]
            assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
            x, _ = S.lsmr(Af, ATf, b, k, lam)
            xs = scipy_lsmr(A, b, damp=lam, atol=0, btol=0, conlim=0, maxiter=k)[0]
            assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_converge_to_least_squares():
    A, b = _random_problem(m=40, n=12, cond=5.0, seed=7)
    Af, ATf = _ops(A)
    x_ls, *_ = np.linalg.lstsq(A, b, rcond=None)
    for fn in (S.cgls, S.lsqr, S.lsmr):
        x, _ = fn(Af, ATf, b, 40)
        assert np.linalg.norm(x - x_ls) <= 1e-10 * np.linalg.norm(x_ls), fn.__name__


@pytest.mark.parametrize("lam", [0.3, 2.0])
def test_damped_normal_equations(lam):
    A, b = _ct_problem(2)
    Af, ATf = _ops(A)
    n = A.shape[1]
    x_t = np.linalg.solve(A.T @ A + lam * lam * np.eye(n), A.T @ b)
    for fn in (S.cgls, S.lsqr, S.lsmr):
        # Converged well inside 100 steps (cond(A^T A + lam^2 I) <= 1e2); run
        # much longer, plain CGLS's recurred residual drifts from b - A x.
        x, _ = fn(Af, ATf, b, 100, lam)
        assert np.linalg.norm(x - x_t) <= 1e-8 * np.linalg.norm(x_t), fn.__name__
    x, _ = S.hybrid_lsqr(Af, ATf, b, 100, lam)
    assert np.linalg.norm(x - x_t) <= 1e-8 * np.linalg.norm(x_t)


def test_cgls_equals_lsqr_and_hybrid_equals_damped():
    A, b = _ct_problem(3)
    Af, ATf = _ops(A)
    for k in (1, 5, 10):
        xc, _ = S.cgls(Af, ATf, b, k)
        xq, _ = S.lsqr(Af, ATf, b, k)
        assert np.linalg.norm(xc - xq) <= 1e-9 * np.linalg.norm(xq)
        for lam in (0.5, 3.0):
            xd, _ = S.lsqr(Af, ATf, b, k, lam)
            xh, _ = S.hybrid_lsqr(Af, ATf, b, k, lam)
            xcd, _ = S.cgls(Af, ATf, b, k, lam)
            assert np.linalg.norm(xh - xd) <= 1e-10 * np.linalg.norm(xd)
            assert np.linalg.norm(xcd - xd) <= 1e-9 * np.linalg.norm(xd)


def test_monotone_and_recurred_norms():
    A, b = _ct_problem(4)
    Af, ATf = _ops(A)
    n = 15
    res_c, res_q, nrm_m = [], [], []
    for k in range(1, n + 1):
        xc, hc = S.cgls(Af, ATf, b, k)
        xq, hq = S.lsqr(Af, ATf, b, k)
        xm, hm = S.lsmr(Af, ATf, b, k)
        rc, rq = np.linalg.norm(b - A @ xc), np.linalg.norm(b - A @ xq)
        rm = np.linalg.norm(A.T @ (b - A @ xm))
        assert abs(hc["res"][-1] - rc) <= 1e-9 * rc
        assert abs(hq["res"][-1] - rq) <= 1e-9 * rq
        assert abs(hm["normal"][-1] - rm) <= 1e-7 * rm
        res_c.append(rc), res_q.append(rq), nrm_m.append(rm)
    assert np.all(np.diff(res_c) <= 1e-12 * res_c[0])
    assert np.all(np.diff(res_q) <= 1e-12 * res_q[0])
    assert np.all(np.diff(nrm_m) <= 1e-12 * nrm_m[0])
    # Damped recurrences against explicit augmented norms.
    lam = 0.8
    xq, hq = S.lsqr(Af, ATf, b, 7, lam)
    aug = math.sqrt(np.linalg.norm(b - A @ xq) ** 2 + lam * lam * np.linalg.norm(xq) ** 2)
    assert abs(hq["res"][-1] - aug) <= 1e-9 * aug
    xm, hm = S.lsmr(Af, ATf, b, 7, lam)
    nrm = np.linalg.norm(A.T @ (b - A @ xm) - lam * lam * xm)
    assert abs(hm["normal"][-1] - nrm) <= 1e-7 * nrm
    xh, hh = S.hybrid_lsqr(Af, ATf, b, 7, lam)
    assert abs(hh["res"][-1] - aug) <= 1e-9 * aug


def test_breakdown_returns_zero():
    A, b = _ct_problem(5)
    Af, ATf = _ops(A)
    zero = np.zeros_like(b)
    for fn in (S.cgls, S.lsqr, S.lsmr):
        x, _ = fn(Af, ATf, zero, 5)
        assert np.all(x == 0.0) and np.all(np.isfinite(x))
    # b orthogonal to range(A): A^T b = 0, alpha_1 = 0.
    Q, _ = np.linalg.qr(np.hstack([A, np.random.default_rng(0).standard_normal((A.shape[0], 1))]))
    bn = Q[:, -1] * (np.linalg.norm(A.T @ Q[:, -1]) < 1e-9)
    if np.linalg.norm(bn) > 0:
        for fn in (S.cgls, S.lsqr, S.lsmr):
            x, _ = fn(Af, ATf, bn, 5)
            assert np.all(np.isfinite(x)) and np.linalg.norm(x) < 1e-6


# ---- hybrid LSQR with a per-iteration parameter choice (Sec. 2.2.2) ---------

def _full_gcv(A, b, lam):
    """GCV of the full Tikhonov problem from its influence matrix
    H = A (A^T A + lam^2 I)^-1 A^T: ||(I - H) b||^2 / tr(I - H)^2."""
    n = A.shape[1]
    H = A @ np.linalg.solve(A.T @ A + lam * lam * np.eye(n), A.T)
    R = np.eye(A.shape[0]) - H
    return float(np.linalg.norm(R @ b) ** 2 / np.trace(R) ** 2)


def test_projected_gcv_equals_full_gcv():
    """With A of size (n+1) x n and k = n Golub-Kahan steps, U_{n+1} is a
    square orthogonal matrix, so the projected GCV function equals the full
    problem's GCV function (residual and trace alike) for every lambda."""
    A, b = _random_problem(m=7, n=6, cond=3.0, seed=4)
    Af, ATf = _ops(A)
    Us, Vs, B, beta1 = S.golub_kahan(Af, ATf, b, 6)
    assert B.shape == (7, 6)
    U = np.array(Us).T
    assert np.abs(U.T @ U - np.eye(7)).max() < 1e-12  # the identity needs an orthogonal U
    s, Q, c = S._projected_svd(B, beta1)
    for lam in (1e-3, 0.02, 0.3, 1.0, 5.0):
        assert S.gcv(s, c, lam) == pytest.approx(_full_gcv(A, b, lam), rel=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gcv_choice_is_the_grid_minimum(seed):
    """The chosen lambda is at least as good as the best of 20001 brute-force
    points over the search range, and never beaten by its neighbours."""
    A, b = _ct_problem(seed)
    Af, ATf = _ops(A)
    for k in (3, 8, 15):
        _, _, B, beta1 = S.golub_kahan(Af, ATf, b, k)
        s, _, c = S._projected_svd(B, beta1)
        lam = S.lambda_gcv(s, c)
        L = math.log10(s[0])
        brute = min(S.gcv(s, c, 10.0 ** g) for g in np.linspace(L - 7.0, L + 1.0, 20001))
        g0 = S.gcv(s, c, lam)
        assert g0 <= brute * (1 + 1e-9)
        assert g0 <= S.gcv(s, c, lam * 1.001) and g0 <= S.gcv(s, c, lam / 1.001)


def test_hybrid_dp_meets_discrepancy():
    """Discrepancy principle: at every iteration where the target residual is
    reachable, the full-space residual ||A x_k - b|| of the returned iterate
    equals nl ||b||; before that, lambda_k = 0 and x_k is the LSQR iterate."""
    A, _ = _random_problem(m=40, n=12, cond=10.0, seed=7)
    rng = np.random.default_rng(7)
    bc = A @ rng.standard_normal(12)
    e = rng.standard_normal(40)
    b = bc + 0.05 * np.linalg.norm(bc) / np.linalg.norm(e) * e
    nl = 0.05 * np.linalg.norm(bc) / np.linalg.norm(b)
    Af, ATf = _ops(A)
    reached = 0
    for k in range(1, 13):
        x, h = S.hybrid_lsqr(Af, ATf, b, k, 0.0, rule="dp", noise_level=nl)
        lam = h["lam"][-1]
        r = np.linalg.norm(A @ x - b)
        U = np.array(S.golub_kahan(Af, ATf, b, k)[0]).T
        orth = np.abs(U.T @ U - np.eye(U.shape[1])).max()
        if lam > 0:
            # ||A x_k - b|| = ||B_k y_k - beta1 e1|| needs U_{k+1} orthonormal,
            # which Golub-Kahan without reorthogonalisation keeps only so long.
            if orth < 1e-8:
                assert r == pytest.approx(nl * np.linalg.norm(b), rel=1e-8)
                reached += 1
        else:
            xl, _ = S.lsqr(Af, ATf, b, k)
            assert np.linalg.norm(x - xl) <= 1e-10 * np.linalg.norm(xl)
            assert r >= nl * np.linalg.norm(b) * (1 - 1e-12)
    assert reached >= 1


def test_hybrid_rules_edge_cases():
    A, b = _random_problem(seed=3)
    Af, ATf = _ops(A)
    # Noise level above 1: every lambda leaves the residual below the target, so the
    # regularisation is infinite and x = 0.
    x, h = S.hybrid_lsqr(Af, ATf, b, 5, 0.0, rule="dp", noise_level=1.5)
    assert np.all(np.isinf(h["lam"])) and not np.any(x)
    assert h["res"][-1] == pytest.approx(np.linalg.norm(b))
    # A fixed lambda reproduces damped LSQR; GCV picks a finite positive value.
    xf, hf = S.hybrid_lsqr(Af, ATf, b, 6, 0.7, rule="fixed")
    xd, _ = S.lsqr(Af, ATf, b, 6, 0.7)
    assert np.linalg.norm(xf - xd) <= 1e-10 * np.linalg.norm(xd)
    _, hg = S.hybrid_lsqr(Af, ATf, b, 6, 0.0, rule="gcv")
    assert np.all(np.isfinite(hg["lam"])) and np.all(hg["lam"] > 0)


# ---- AB- and BA-GMRES (Sec. 2.1.4) ------------------------------------------

def test_ab_ba_gmres_with_matched_backprojector():
    """With B = A^T, AB-GMRES minimises ||b - A x|| over K_k(A^T A, A^T b)
    (LSQR's iterate) and BA-GMRES minimises ||A^T (b - A x)|| over the same
    space (LSMR's iterate)."""
    A, b = _ct_problem(5)
    Af, ATf = _ops(A)
    for k in (1, 3, 7):
        xa, ha = S.ab_gmres(Af, ATf, b, k)
        xq, hq = S.lsqr(Af, ATf, b, k)
        assert np.linalg.norm(xa - xq) <= 1e-9 * np.linalg.norm(xq)
        assert ha["res"][-1] == pytest.approx(np.linalg.norm(b - A @ xq), rel=1e-9)
        xb, hb = S.ba_gmres(Af, ATf, b, k)
        xm, _ = S.lsmr(Af, ATf, b, k)
        assert np.linalg.norm(xb - xm) <= 1e-9 * np.linalg.norm(xm)
        assert hb["res"][-1] == pytest.approx(np.linalg.norm(A.T @ (b - A @ xm)), rel=1e-9)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_gmres_krylov_optimality_unmatched(k):
    """With a B that is not A^T, the iterates are the explicit minimisers over
    explicitly built Krylov spaces: x = B y, y in K_k(AB, b) minimising
    ||b - A B y|| (AB); x in K_k(BA, Bb) minimising ||B(b - A x)|| (BA)."""
    A, b = _ct_problem(6)
    rng = np.random.default_rng(k)
    Bm = A.T * (1.0 + 0.2 * rng.standard_normal(A.T.shape))  # a perturbed back projector
    Af, Bf = (lambda x: A @ x), (lambda y: Bm @ y)
    xa, _ = S.ab_gmres(Af, Bf, b, k)
    K = [b]
    for _ in range(k - 1):
        K.append(A @ (Bm @ K[-1]))
    Q, _ = np.linalg.qr(np.array(K).T)
    y, *_ = np.linalg.lstsq(A @ Bm @ Q, b, rcond=None)
    xr = Bm @ (Q @ y)
    assert np.linalg.norm(xa - xr) <= 1e-8 * np.linalg.norm(xr)
    xb, _ = S.ba_gmres(Af, Bf, b, k)
    K = [Bm @ b]
    for _ in range(k - 1):
        K.append(Bm @ (A @ K[-1]))
    Q, _ = np.linalg.qr(np.array(K).T)
    y, *_ = np.linalg.lstsq(Bm @ A @ Q, Bm @ b, rcond=None)
    assert np.linalg.norm(xb - Q @ y) <= 1e-8 * np.linalg.norm(Q @ y)


# ---- SIRT and OS-SART (the comparison methods of Sec. 3) --------------------

def _positive_problem(m=40, n=12, seed=11):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.1, 1.0, (m, n)), rng


def test_sirt_fixed_point_is_weighted_least_squares():
    """SIRT's fixed point solves A^T W (b - A x) = 0: the least-squares
    solution in the W-weighted norm, here found by lstsq on W^(1/2) A."""
    A, rng = _positive_problem()
    b = rng.uniform(0.5, 2.0, A.shape[0])
    x, h = S.sirt(*_ops(A), b, 4000)
    w = 1.0 / A.sum(1)
    ref, *_ = np.linalg.lstsq(np.sqrt(w)[:, None] * A, np.sqrt(w) * b, rcond=None)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def test_os_sart_one_subset_is_sirt_and_solves_consistent_systems():
    A, rng = _positive_problem(seed=12)
    xt = rng.uniform(0.0, 1.0, A.shape[1])
    b = A @ xt
    Af, ATf = _ops(A)
    x1, h1 = S.os_sart([(Af, ATf)], [b], 30)
    xs, hs = S.sirt(Af, ATf, b, 30)
    assert np.linalg.norm(x1 - xs) <= 1e-12 * np.linalg.norm(xs)
    np.testing.assert_allclose(h1["res"], hs["res"], rtol=1e-12)
    # Four interleaved subsets of the rows: the consistent system's solution.
    parts = [np.arange(s, A.shape[0], 4) for s in range(4)]
    subs = [((lambda x, P=P: A[P] @ x), (lambda y, P=P: A[P].T @ y)) for P in parts]
    x4, h4 = S.os_sart(subs, [b[P] for P in parts], 3000)
    assert np.linalg.norm(x4 - xt) <= 1e-6 * np.linalg.norm(xt)
    assert h4["res"][-1] < 1e-6 * h4["res"][0]


def test_explicit_residual_stop_rule_by_hand():
    """The stop rule (Sec. 3.1.1): residual norms 3, 2, 2, 2.5, 1 stop at the
    fourth iterate (the first strict increase) and return the third; a
    sequence that never grows returns its last iterate."""
    b = np.array([3.0, 0.0])
    A = lambda x: x  # noqa: E731
    its = [b - np.array([r, 0.0]) for r in (3.0, 2.0, 2.0, 2.5, 1.0)]
    k, x, res = S.explicit_residual_stop(A, b, its)
    assert k == 3 and x is its[2]
    np.testing.assert_allclose(res, [3.0, 2.0, 2.0, 2.5])
    k, x, res = S.explicit_residual_stop(A, b, its[:3] + its[4:])
    assert k is None and x is its[-1] and len(res) == 4


def test_stop_rule_quiet_for_exact_cgls_and_fires_for_a_mismatched_adjoint():
    """Exact-arithmetic CGLS minimises ||b - A x|| over nested spaces, so the
    rule never fires; with a back projector that is not A^T (the situation
    Sec. 3.1.2 blames for growing residuals) it does."""
    rng = np.random.default_rng(5)
    M = rng.standard_normal((40, 25))
    b = rng.standard_normal(40)
    A, AT = (lambda x: M @ x), (lambda y: M.T @ y)
    its = [S.cgls(A, AT, b, k)[0] for k in range(1, 26)]
    k, _, res = S.explicit_residual_stop(A, b, its)
    assert k is None and np.all(np.diff(res) <= 1e-12 * res[0])
    E = rng.standard_normal((25, 40))
    B = lambda y: M.T @ y + 0.6 * (E @ y)  # noqa: E731
    its = [S.cgls(A, B, b, k)[0] for k in range(1, 26)]
    k, x, res = S.explicit_residual_stop(A, b, its)
    assert k is not None and res[k] > res[k - 1] and x is its[k - 1]
