"""FP64 Krylov solvers of the oracle: CGLS, LSQR, LSMR, hybrid LSQR, IRN-TV.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every solver is matrix-free: it takes callables ``A(x)`` and ``AT(y)`` that
apply the operator and its transpose, works in float64 NumPy, starts from
x0 = 0 unless told otherwise, and runs a fixed number of iterations.  Each
returns ``(x, hist)`` where ``hist`` holds per-iteration FP64 scalars.

Sources (the paper states the objectives; the recurrences are those of the
works it cites for each method).  Equations are named by their labels:
  * CGLS      -- Sec. 2.1.1, eq. (lest_squares_projected): CG on the normal
                 equations (Hestenes and Stiefel); with damping lambda it solves
                 the Tikhonov problem, eq. (Tikhonov), via the augmented system
                 of eq. (Tikhonov_augmented).
  * LSQR      -- Sec. 2.1.2, eq. (proj_LSQR): Golub-Kahan bidiagonalisation and
                 the short recurrences of Paige and Saunders (1982), damped form.
  * LSMR      -- Sec. 2.1.3, eq. (proj_LSMR): minimises ||A^T r_k|| over the
                 same Krylov space (Fong and Saunders 2011), damped form.
  * hybrid    -- Sec. 2.2.1, eq. (hybrid_LSQR): Tikhonov on the projected
                 problem, solved through the SVD of the stored bidiagonal
                 matrix, with lambda fixed or chosen at every iteration by
                 GCV or the discrepancy principle (Sec. 2.2.2).
  * AB-/BA-GMRES -- Sec. 2.1.4: GMRES on A B (B a right preconditioner) or
                 on B A (left), for a back projector B that need not be A^T.
  * SIRT, OS-SART -- the algebraic methods of the comparisons (Sec. 3): the
                 simultaneous update with inverse row and column sums, and its
                 ordered-subset form.
  * stop rule -- Sec. 3.1.1 and 3.1.2: stop when the residual computed
                 from the iterate grows between two iterations.
  * IRN-TV    -- Sec. 2.3, eqs. (TV), (TV_reweighted), (TV_approx) and
                 Sec. 2.3.1: reweighted quadratic majorants of isotropic TV, each
                 solved by CGLS on [A; lam L D].
  * hybrid fLSQR-TV -- Sec. 2.3.2, eq. (TV_standard_form): the same weights
                 as a changing right preconditioner (the A-weighted
                 pseudoinverse of L D) in a flexible Golub-Kahan process, with
                 the hybrid projected Tikhonov solve.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return float(np.dot(a.ravel(), b.ravel()))


def _nrm(a):
    return float(np.sqrt(np.dot(a.ravel(), a.ravel())))


# --------------------------------------------------------------------------
# CGLS (Sec. 2.1.1): x_k minimises ||A x - b|| over K_k(A^T A, A^T b).
# --------------------------------------------------------------------------
def cgls(A, AT, b, n_iter, lam=0.0, x0=None):
    """Conjugate gradients on (A^T A + lam^2 I) x = A^T b.

    hist: 'res' = ||b - A x_k|| (the data residual, recurred), 'res_damped' =
    sqrt(||r||^2 + lam^2 ||x||^2), 'normal' = ||A^T r_k - lam^2 x_k||,
    'alpha', 'beta'.
    """
    b = np.asarray(b, dtype=np.float64)
    lam2 = float(lam) ** 2
    if x0 is None:
        x = np.zeros_like(AT(b))
        r = b.copy()
    else:
        x = np.array(x0, dtype=np.float64)
        r = b - A(x)
    s = AT(r) - lam2 * x
    p = s.copy()
    gamma = _dot(s, s)
    hist = {"res": [], "res_damped": [], "normal": [], "alpha": [], "beta": []}
    for _ in range(n_iter):
        if gamma == 0.0:
            break
        q = A(p)
        delta = _dot(q, q) + lam2 * _dot(p, p)
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        s = AT(r) - lam2 * x
        gamma_new = _dot(s, s)
        beta = gamma_new / gamma
        gamma = gamma_new
        p = s + beta * p
        rn = _nrm(r)
        hist["res"].append(rn)
        hist["res_damped"].append(np.sqrt(rn * rn + lam2 * _dot(x, x)))
        hist["normal"].append(np.sqrt(gamma))
        hist["alpha"].append(alpha)
        hist["beta"].append(beta)
    return x, {k: np.asarray(v) for k, v in hist.items()}


# --------------------------------------------------------------------------
# Golub-Kahan bidiagonalisation (Sec. 2.1.2): A V_k = U_{k+1} B_k.
# --------------------------------------------------------------------------
def _normalise(w):
    n = _nrm(w)
    return (w / n if n > 0.0 else w * 0.0), n


def lsqr(A, AT, b, n_iter, lam=0.0):
    """LSQR with damping ``lam`` (Paige and Saunders, Sec. 2.1.2 / Sec. 2.2).

    Iterates x_k minimise ||[A; lam I] x - [b; 0]|| over K_k.  hist: 'res'
    (recurred ||[b;0] - [A;lam I] x_k||), 'alpha', 'beta' (the bidiagonal
    entries alpha_{k+1}, beta_{k+1} produced in iteration k).
    """
    b = np.asarray(b, dtype=np.float64)
    u, beta = _normalise(b.copy())
    v, alpha = _normalise(AT(u))
    x = np.zeros_like(v)
    w = v.copy()
    phibar, rhobar = beta, alpha
    psi_sq = 0.0
    hist = {"res": [], "alpha": [], "beta": []}
    for _ in range(n_iter):
        if alpha == 0.0 or beta == 0.0:
            break
        # Bidiagonalisation: beta_{k+1} u_{k+1} = A v_k - alpha_k u_k, then
        # alpha_{k+1} v_{k+1} = A^T u_{k+1} - beta_{k+1} v_k.
        u, beta = _normalise(A(v) - alpha * u)
        v, alpha = _normalise(AT(u) - beta * v)
        # Rotation that folds the damping row lam into rhobar.
        rhohat = np.hypot(rhobar, lam)
        c1, s1 = rhobar / rhohat, lam / rhohat
        psi = s1 * phibar
        phibar = c1 * phibar
        psi_sq += psi * psi
        # Rotation that eliminates beta_{k+1} from the bidiagonal.
        rho = np.hypot(rhohat, beta)
        c, s = rhohat / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        hist["res"].append(np.sqrt(phibar * phibar + psi_sq))
        hist["alpha"].append(alpha)
        hist["beta"].append(beta)
    return x, {k: np.asarray(v) for k, v in hist.items()}


def lsmr(A, AT, b, n_iter, lam=0.0):
    """LSMR with damping ``lam`` (Fong and Saunders, Sec. 2.1.3).

    Iterates x_k minimise ||A_lam^T r_k|| over K_k, where A_lam = [A; lam I]
    and r_k = [b; 0] - A_lam x_k.  hist: 'normal' = recurred ||A_lam^T r_k||
    (= |zetabar_{k+1}|), 'alpha', 'beta'.
    """
    b = np.asarray(b, dtype=np.float64)
    u, beta = _normalise(b.copy())
    v, alpha = _normalise(AT(u))
    x = np.zeros_like(v)
    h = v.copy()
    hbar = np.zeros_like(v)
    alphabar = alpha
    zetabar = alpha * beta
    rho_old, rhobar_old = 1.0, 1.0
    cbar, sbar = 1.0, 0.0
    hist = {"normal": [], "alpha": [], "beta": []}
    for _ in range(n_iter):
        if alpha == 0.0 or beta == 0.0:
            break
        u, beta = _normalise(A(v) - alpha * u)
        v, alpha = _normalise(AT(u) - beta * v)
        # Fold the damping into alphabar (first rotation of the damped problem).
        alphahat = np.hypot(alphabar, lam)
        # Rotation P_k: eliminate beta_{k+1} from the lower bidiagonal.
        rho = np.hypot(alphahat, beta)
        c, s = alphahat / rho, beta / rho
        theta_next = s * alpha
        alphabar = c * alpha
        # Rotation Pbar_k: turn R_k^T into lower bidiagonal form.
        thetabar = sbar * rho
        rhobar = np.hypot(cbar * rho, theta_next)
        cbar_new = cbar * rho / rhobar
        sbar = theta_next / rhobar
        zeta = cbar_new * zetabar
        zetabar = -sbar * zetabar
        cbar = cbar_new
        # Vector updates.
        hbar = h - (thetabar * rho / (rho_old * rhobar_old)) * hbar
        x = x + (zeta / (rho * rhobar)) * hbar
        h = v - (theta_next / rho) * h
        rho_old, rhobar_old = rho, rhobar
        hist["normal"].append(abs(zetabar))
        hist["alpha"].append(alpha)
        hist["beta"].append(beta)
    return x, {k: np.asarray(v) for k, v in hist.items()}


# --------------------------------------------------------------------------
# Hybrid LSQR with a fixed lambda (Sec. 2.2.1, eq. (hybrid_LSQR)).
# --------------------------------------------------------------------------
def golub_kahan(A, AT, b, k):
    """k steps of GK: returns (U (k+1 vectors), V (k vectors), B (k+1 x k), beta1).

    A V_k = U_{k+1} B_k with B_k lower bidiagonal: B[i, i] = alpha_{i+1},
    B[i+1, i] = beta_{i+2}.  Stops early on breakdown.
    """
    b = np.asarray(b, dtype=np.float64)
    u, beta1 = _normalise(b.copy())
    v, alpha = _normalise(AT(u))
    Us, Vs = [u], []
    alphas, betas = [], []
    for _ in range(k):
        if alpha == 0.0:
            break
        Vs.append(v)
        alphas.append(alpha)
        u, beta = _normalise(A(v) - alpha * u)
        Us.append(u)
        betas.append(beta)
        if beta == 0.0:
            break
        v, alpha = _normalise(AT(u) - beta * v)
    kk = len(Vs)
    B = np.zeros((kk + 1, kk))
    for i in range(kk):
        B[i, i] = alphas[i]
        B[i + 1, i] = betas[i]
    return Us, Vs, B, beta1


def _projected_svd(Bk, beta1):
    """SVD of the projected matrix: singular values s (k, descending), right
    singular vectors Q (k x k, columns), and c = P^T (beta1 e1) (k+1 entries;
    c[k] is the part of beta1 e1 outside the range of B_k)."""
    P, s, Qt = np.linalg.svd(Bk, full_matrices=True)
    return s, Qt.T, beta1 * P[0, :]


def _filters(s, lam):
    """Tikhonov filter factors s^2 / (s^2 + lam^2); 0 where s = 0."""
    s2 = s * s
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(s2 > 0, s2 / (s2 + lam * lam), 0.0)
    return f


def projected_residual2(s, c, lam):
    """||(I - B_k B_k^dagger(lam)) beta1 e1||^2, the squared data residual of
    the projected Tikhonov solution (equal to ||A x_k - b||^2 while U_{k+1} has
    orthonormal columns)."""
    k = s.size
    f = _filters(s, lam)
    return float(np.sum(((1.0 - f) * c[:k]) ** 2) + c[k] ** 2)


def gcv(s, c, lam):
    """GCV function of the projected problem (Sec. 2.2.2, GCV equation), with
    B^dagger(lam) = (B^T B + lam^2 I)^-1 B^T: the squared residual over the
    squared trace of I_{k+1} - B B^dagger(lam) = 1 + sum_i (1 - f_i)."""
    f = _filters(s, lam)
    return projected_residual2(s, c, lam) / (1.0 + float(np.sum(1.0 - f))) ** 2


GCV_GRID = 81          # log10 lambda grid: sigma_max * 10^[-7, 1], 0.1 decade apart
GCV_GOLDEN_STEPS = 60  # golden-section steps on the bracketing grid cells
DP_BISECT_STEPS = 64   # bisection steps on log10 lambda in sigma_max * 10^[-12, 8]


def lambda_gcv(s, c):
    """Minimiser of the projected GCV function: the smallest value on a
    log-spaced grid, refined by golden-section search over its two grid
    cells (the paper states the minimisation, not how it is carried out)."""
    if s.size == 0 or s[0] == 0.0:
        return 0.0
    L = np.log10(s[0])
    grid = L - 7.0 + 8.0 * np.arange(GCV_GRID) / (GCV_GRID - 1)
    G = [gcv(s, c, 10.0 ** g) for g in grid]
    j = int(np.argmin(G))
    a, b = grid[max(j - 1, 0)], grid[min(j + 1, GCV_GRID - 1)]
    r = (np.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = b - r * (b - a), a + r * (b - a)
    f1, f2 = gcv(s, c, 10.0 ** x1), gcv(s, c, 10.0 ** x2)
    for _ in range(GCV_GOLDEN_STEPS):
        if f1 <= f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - r * (b - a)
            f1 = gcv(s, c, 10.0 ** x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + r * (b - a)
            f2 = gcv(s, c, 10.0 ** x2)
    return float(10.0 ** (0.5 * (a + b)))


def lambda_dp(s, c, target):
    """Discrepancy principle (Sec. 2.2.2, DP equations): the lambda at which
    the projected squared residual equals target = (nl ||b||)^2.  The
    residual grows with lambda from c_k^2 (lambda = 0) to beta1^2, so: 0 when
    even lambda = 0 leaves a residual at or above the target, +inf when the
    target is at or above ||b||^2, else the root by bisection on log10
    lambda."""
    k = s.size
    if k == 0 or s[0] == 0.0:
        return 0.0
    if c[k] ** 2 >= target:
        return 0.0
    if float(np.sum(c * c)) <= target:
        return float("inf")
    L = np.log10(s[0])
    lo, hi = L - 12.0, L + 8.0
    for _ in range(DP_BISECT_STEPS):
        mid = 0.5 * (lo + hi)
        if projected_residual2(s, c, 10.0 ** mid) < target:
            lo = mid
        else:
            hi = mid
    return float(10.0 ** (0.5 * (lo + hi)))


def projected_tikhonov(Bk, beta1, rule, lam, noise_level=None):
    """Tikhonov solution of the projected problem
    min ||Bk y - beta1 e1||^2 + lam_k^2 ||y||^2 for a (k+1) x k matrix Bk.

    lam_k is ``lam`` (rule "fixed"), the GCV minimiser (rule "gcv"), or the
    discrepancy-principle root for the relative noise level ``noise_level``
    (rule "dp"), from the SVD of Bk.  y = Q diag(s / (s^2 + lam_k^2)) c[:k].
    Returns (y, lam_k, res) with res = ||[beta1 e1; 0] - [Bk; lam_k I] y||
    (beta1 when lam_k is infinite and y = 0).
    """
    k = Bk.shape[1]
    s, Q, c = _projected_svd(Bk, beta1)
    if rule == "gcv":
        lk = lambda_gcv(s, c)
    elif rule == "dp":
        lk = lambda_dp(s, c, (noise_level * beta1) ** 2)
    else:
        lk = float(lam)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = np.where(s > 0, s / (s * s + lk * lk), 0.0) if np.isfinite(lk) else np.zeros_like(s)
    y = Q @ (g * c[:k])
    if not np.isfinite(lk):
        return y, lk, float(beta1)
    return y, lk, float(np.sqrt(projected_residual2(s, c, lk) + lk * lk * float(np.dot(y, y))))


def hybrid_lsqr(A, AT, b, n_iter, lam, rule="fixed", noise_level=None):
    """x_k = V_k y_k, y_k = argmin ||beta1 e1 - B_k y||^2 + lam_k^2 ||y||^2
    (Sec. 2.2.1, eq. (hybrid_LSQR)).

    lam_k is recomputed at every k by ``projected_tikhonov`` from the SVD of
    B_k (rule "fixed", "gcv" or "dp"; ``noise_level`` = ||e|| / ||b||).
    hist: 'res' = ||[beta1 e1; 0] - [B_k; lam_k I] y_k|| (the projected
    Tikhonov residual, equal to the augmented-system residual while U_{k+1}
    is orthonormal), 'lam' = lam_k, 'y' = the last y_k.
    """
    if rule not in ("fixed", "gcv", "dp"):
        raise ValueError(rule)
    Us, Vs, B, beta1 = golub_kahan(A, AT, b, n_iter)
    hist = {"res": [], "lam": []}
    y = np.zeros(0)
    for k in range(1, B.shape[1] + 1):
        y, lk, res = projected_tikhonov(B[: k + 1, :k], beta1, rule, lam, noise_level)
        hist["res"].append(res)
        hist["lam"].append(lk)
    x = np.zeros_like(Vs[0]) if Vs else np.zeros_like(AT(np.asarray(b, dtype=np.float64)))
    for i, yi in enumerate(y):
        x = x + yi * Vs[i]
    hist["y"] = y
    hist["res"] = np.asarray(hist["res"])
    hist["lam"] = np.asarray(hist["lam"])
    return x, hist


# --------------------------------------------------------------------------
# AB- and BA-GMRES with a back projector B (Sec. 2.1.4).
# --------------------------------------------------------------------------
def _arnoldi(op, r0, k):
    """k steps of Arnoldi (modified Gram-Schmidt) on ``op`` from r0.

    Returns (V, H, beta) with V the basis vectors (up to k+1), H the
    (j+1) x j upper Hessenberg matrix of the steps taken, beta = ||r0||;
    stops early when a new vector has zero norm.
    """
    r0 = np.asarray(r0, dtype=np.float64)
    v, beta = _normalise(r0.copy())
    V = [v]
    H = np.zeros((k + 1, k))
    j = 0
    for j in range(k):
        if beta == 0.0:
            return V[:1], H[:1, :0], beta
        w = np.asarray(op(V[j]), dtype=np.float64).copy()
        for i in range(j + 1):
            H[i, j] = _dot(w, V[i])
            w = w - H[i, j] * V[i]
        h = _nrm(w)
        H[j + 1, j] = h
        if h == 0.0:
            return V, H[: j + 2, : j + 1], beta
        V.append(w / h)
    return V, H[: k + 1, :k], beta


def _gmres_coeffs(H, beta):
    """y = argmin ||beta e1 - H y|| (dense FP64 least squares); and the residual."""
    rhs = np.zeros(H.shape[0])
    rhs[0] = beta
    if H.shape[1] == 0:
        return np.zeros(0), beta
    y, *_ = np.linalg.lstsq(H, rhs, rcond=None)
    return y, float(np.linalg.norm(rhs - H @ y))


def _gmres_run(op, r0, n_iter):
    """Arnoldi once for n_iter steps; the GMRES iterate of step k uses only
    the leading (k+1) x k block of H.  Returns (V, y of the last step, hist)."""
    V, H, beta = _arnoldi(op, r0, n_iter)
    hist = {"res": []}
    y = np.zeros(0)
    for k in range(1, n_iter + 1):
        kk = min(k, H.shape[1])
        y, res = _gmres_coeffs(H[: kk + 1, :kk], beta)
        hist["res"].append(res)
    hist["res"] = np.asarray(hist["res"])
    return V, y, hist


def ab_gmres(A, B, b, n_iter):
    """AB-GMRES: x_k = B y_k with y_k = argmin ||b - A B y|| over K_k(AB, b)
    (GMRES on AB, B a right preconditioner).  hist 'res' = ||b - A x_k||
    (the GMRES residual of iteration k).  With B = A^T this is LSQR."""
    b = np.asarray(b, dtype=np.float64)
    V, y, hist = _gmres_run(lambda z: A(B(z)), b, n_iter)
    z = sum(yi * V[i] for i, yi in enumerate(y)) if len(y) else np.zeros_like(b)
    return B(z), hist


def ba_gmres(A, B, b, n_iter):
    """BA-GMRES: x_k = argmin ||B (b - A x)|| over K_k(BA, B b) (GMRES on BA,
    B a left preconditioner).  hist 'res' = ||B (b - A x_k)||.  With B = A^T
    this is LSMR."""
    r0 = B(np.asarray(b, dtype=np.float64))
    V, y, hist = _gmres_run(lambda z: B(A(z)), r0, n_iter)
    x = sum(yi * V[i] for i, yi in enumerate(y)) if len(y) else np.zeros_like(r0)
    return x, hist


# --------------------------------------------------------------------------
# SIRT and OS-SART, the algebraic baselines the paper compares with (Sec. 3).

# ---------------------------------------------------------------------------
# Explicit-residual stop rule (Sec. 3.1.1 and 3.1.2): after each iteration the
# residual ||b - A x_k|| is computed from the iterate itself, not recurred; the
# first time it is larger than at the previous iteration the run stops and
# returns the previous iterate.  Reading: the comparison starts with the pair
# (x_1, x_2); x_0 = 0 is not compared.


def explicit_residual_stop(A, b, iterates):
    """Apply the rule to the iterates x_1..x_n.

    Returns (k, x, res): k is the 0-based index of the first iterate whose
    explicit residual exceeds its predecessor's (None if none does), x the
    iterate returned (x_{k-1} in that 0-based numbering, else the last one) and
    res the explicit residual norms up to and including iterate k.
    """
    res = []
    for k, x in enumerate(iterates):
        res.append(_nrm(b - A(x)))
        if k > 0 and res[k] > res[k - 1]:
            return k, iterates[k - 1], np.asarray(res)
    return None, iterates[-1], np.asarray(res)


# --------------------------------------------------------------------------
def _inv_or_zero(v):
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    nz = v != 0
    out[nz] = 1.0 / v[nz]
    return out


def sirt(A, AT, b, n_iter, lam=1.0):
    """SIRT: x_{k+1} = x_k + lam V A^T W (b - A x_k) from x_0 = 0, with
    W = diag(1 / A 1) (inverse ray lengths) and V = diag(1 / A^T 1) (inverse
    column sums), 0 where a sum vanishes.  hist 'res' = ||b - A x_k|| before
    update k+1 (the explicit residual of the iterate the step starts from)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(np.asarray(AT(b), dtype=np.float64))
    W = _inv_or_zero(A(np.ones_like(x)))
    V = _inv_or_zero(AT(np.ones_like(b)))
    hist = {"res": []}
    for _ in range(n_iter):
        r = b - A(x)
        hist["res"].append(_nrm(r))
        x = x + lam * V * AT(W * r)
    hist["res"] = np.asarray(hist["res"])
    return x, hist


def os_sart(subsets, b_subsets, n_iter, lam=1.0):
    """OS-SART: one iteration sweeps the ordered subsets s = 1..m of the
    projection data, x <- x + lam V_s A_s^T W_s (b_s - A_s x) with the SIRT
    weights of each subset's operator (A_s, A_s^T) = subsets[s].  x_0 = 0.
    hist 'res' = sqrt(sum_s ||b_s - A_s x||^2), each term taken just before
    subset s updates x (no extra projection)."""
    bs = [np.asarray(bb, dtype=np.float64) for bb in b_subsets]
    A0, AT0 = subsets[0]
    x = np.zeros_like(np.asarray(AT0(bs[0]), dtype=np.float64))
    Ws = [_inv_or_zero(A(np.ones_like(x))) for A, _ in subsets]
    Vs = [_inv_or_zero(AT(np.ones_like(bb))) for (_, AT), bb in zip(subsets, bs)]
    hist = {"res": []}
    for _ in range(n_iter):
        r2 = 0.0
        for (A, AT), bb, W, V in zip(subsets, bs, Ws, Vs):
            r = bb - A(x)
            r2 += _nrm(r) ** 2
            x = x + lam * V * AT(W * r)
        hist["res"].append(float(np.sqrt(r2)))
    hist["res"] = np.asarray(hist["res"])
    return x, hist


# --------------------------------------------------------------------------
# Isotropic TV and its IRN majorants (Sec. 2.3).
# --------------------------------------------------------------------------
def grad(x):
    """D x: forward differences along x, y, z (unit spacing, Neumann).

    ``x`` has shape (nz, ny, nx); returns shape (3, nz, ny, nx) with the x,
    y, z components; the difference at the last index of each axis is 0.
    """
    g = np.zeros((3,) + x.shape)
    g[0, :, :, :-1] = x[:, :, 1:] - x[:, :, :-1]
    g[1, :, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    g[2, :-1, :, :] = x[1:, :, :] - x[:-1, :, :]
    return g


def grad_T(g):
    """D^T g, the exact adjoint of ``grad``."""
    out = np.zeros(g.shape[1:])
    gx, gy, gz = g[0], g[1], g[2]
    out[:, :, :-1] -= gx[:, :, :-1]
    out[:, :, 1:] += gx[:, :, :-1]
    out[:, :-1, :] -= gy[:, :-1, :]
    out[:, 1:, :] += gy[:, :-1, :]
    out[:-1, :, :] -= gz[:-1, :, :]
    out[1:, :, :] += gz[:-1, :, :]
    return out


def tv(x):
    """Isotropic TV (eq. (TV)): sum over voxels of the gradient's 2-norm."""
    g = grad(x)
    return float(np.sum(np.sqrt(np.sum(g * g, axis=0))))


def irn_weights(x, eps):
    """IRN weights L = diag(w^{-1/2}) with w_i = sqrt(||(D x)_i||^2 + eps^2).

    Returned as the per-voxel factor w^{-1/2} (shape (nz, ny, nx)); the same
    factor multiplies all three gradient components of a voxel.
    """
    g = grad(x)
    w = np.sqrt(np.sum(g * g, axis=0) + eps * eps)
    return 1.0 / np.sqrt(w)


def irn_tv_cgls(A, AT, b, shape, n_outer, n_inner, lam, eps):
    """IRN-TV with inner CGLS (Sec. 2.3.1).

    Outer iteration 0 uses L = I; outer iteration k >= 1 uses the weights of
    the previous outer iterate.  Each outer iteration runs ``n_inner`` CGLS
    steps on K = [A; lam L D] with right-hand side [b; 0], restarted from the
    current iterate (a new Krylov space each time).  hist: 'res' = data
    residual ||b - A x|| after every inner step, 'tv' after each outer step.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(shape)
    hist = {"res": [], "tv": []}
    for k in range(n_outer):
        Lw = np.ones(shape) if k == 0 else irn_weights(x, eps)

        def K(z, Lw=Lw):
            return (A(z), lam * Lw[None] * grad(z))

        def KT(r, Lw=Lw):
            r1, r2 = r
            return AT(r1) + lam * grad_T(Lw[None] * r2)

        # CGLS on the stacked system, with stacked residual (r1, r2).
        q1, q2 = K(x)
        r1, r2 = b - q1, -q2
        s = KT((r1, r2))
        p = s.copy()
        gamma = _dot(s, s)
        for _ in range(n_inner):
            if gamma == 0.0:
                break
            q1, q2 = K(p)
            delta = _dot(q1, q1) + _dot(q2, q2)
            alpha = gamma / delta
            x = x + alpha * p
            r1 = r1 - alpha * q1
            r2 = r2 - alpha * q2
            s = KT((r1, r2))
            gamma_new = _dot(s, s)
            beta = gamma_new / gamma
            gamma = gamma_new
            p = s + beta * p
            hist["res"].append(_nrm(r1))
        hist["tv"].append(tv(x))
    return x, {k: np.asarray(v) for k, v in hist.items()}


# ---------------------------------------------------------------------------
# Hybrid fLSQR-TV (Sec. 2.3.2, eq. (TV_standard_form)).
#
# Each problem of the IRN sequence, eq. (TV_approx) with L = L^(k), is put in
# standard form with the A-weighted pseudoinverse of L D:
#     x = x0 + (L D)_A^dagger ybar,  (L D)_A^dagger = E (L D)^dagger,
# where the null space of L D is the constants (D x = 0 only for constant x on
# a connected grid, and L is a positive diagonal), so with a = A 1:
#     x0 = 1 (a^T b) / (a^T a),  bbar = b - A x0,
#     E z = z - 1 (a^T A z) / (a^T a)   (the oblique projector I - (A N)^dagger A
#                                        restricted to N = span{1}),
# and (L D)^dagger v = K^dagger D^T L v with K = D^T L^2 D (a weighted
# Neumann Laplacian, SPD on the complement of the constants).  Reading: K^dagger
# is applied by ``n_inner`` CG steps from zero (the right-hand sides are
# orthogonal to the constants, so the iterates stay there).  The changing
# preconditioner P_k = E (L^(k) D)^dagger enters a flexible Golub-Kahan process:
#     v_k  = P_k^T A^T u_k orthonormalised against v_1..v_{k-1} (gradient space),
#     z_k  = P_k v_k,
#     A z_k = sum_{i <= k+1} M[i, k] u_i  (u_{k+1} orthonormalised),
# so A Z_k = U_{k+1} M_k with M_k upper Hessenberg, and
#     x_k = x0 + Z_k y_k,  y_k = argmin ||M_k y - beta1 e1||^2 + lam_k^2 ||y||^2
# (||y|| = ||V_k y||, the standard-form penalty).  L^(1) = I and L^(k+1) are the
# IRN weights of x_k (reweighted at every iteration).
# ---------------------------------------------------------------------------


def weighted_laplacian(w2, s):
    """K s = D^T (w2 D s) with w2 = L^2 per voxel (all three components)."""
    return grad_T(w2[None] * grad(s))


def cg_weighted_laplacian(w2, rhs, n_inner):
    """``n_inner`` CG steps on K t = rhs from t = 0 (Hestenes-Stiefel CG) on
    the complement of the constants, where K is SPD: the residual has its mean
    removed at every step, so rounding cannot feed the null space of K (which
    would make the system inconsistent and CG diverge once converged).  Stops
    early when the residual vanishes."""
    t = np.zeros_like(rhs)
    r = rhs - np.mean(rhs)
    p = r.copy()
    gamma = _dot(r, r)
    for _ in range(n_inner):
        if gamma == 0.0:
            break
        q = weighted_laplacian(w2, p)
        alpha = gamma / _dot(p, q)
        t = t + alpha * p
        r = r - alpha * q
        r = r - np.mean(r)
        gamma_new = _dot(r, r)
        p = r + (gamma_new / gamma) * p
        gamma = gamma_new
    return t


def hybrid_flsqr_tv(A, AT, b, shape, n_iter, lam, eps, n_inner, rule="fixed", noise_level=None, reweight=True):
    """Hybrid fLSQR with TV weights (Sec. 2.3.2), as read above.

    ``lam``/``rule``/``noise_level`` choose lam_k on the projected problem as
    in hybrid LSQR; ``n_inner`` CG steps apply each pseudoinverse;
    ``reweight=False`` keeps L = I throughout (then the method is hybrid LSQR
    with full reorthogonalisation on the standard-form problem of
    min ||A x - b||^2 + lam^2 ||D x||^2).  Returns (x, hist) with hist 'res'
    (projected Tikhonov residual per iteration), 'lam' (lam_k), and the
    process's 'U', 'V', 'Z', 'M' for the tests.
    """
    if rule not in ("fixed", "gcv", "dp"):
        raise ValueError(rule)
    b = np.asarray(b, dtype=np.float64)
    a = A(np.ones(shape))
    ca = _dot(a, a)
    c0 = _dot(a, b) / ca if ca > 0.0 else 0.0
    x0 = np.full(shape, c0)
    g = AT(a)
    bbar = b - c0 * a

    def E(z):
        return z - (_dot(g, z) / ca if ca > 0.0 else 0.0)

    def ET(w):
        return w - g * (float(np.sum(w)) / ca) if ca > 0.0 else w

    u, beta1 = _normalise(bbar)
    U, V, Z = [u], [], []
    M = np.zeros((n_iter + 1, n_iter))
    hist = {"res": [], "lam": []}
    x = x0.copy()
    for k in range(n_iter):
        if beta1 == 0.0:
            break
        Lw = irn_weights(x, eps) if (reweight and k > 0) else np.ones(shape)
        w2 = Lw * Lw
        v = Lw[None] * grad(cg_weighted_laplacian(w2, ET(AT(U[k])), n_inner))
        for vi in V:
            v = v - _dot(v, vi) * vi
        v, tkk = _normalise(v)
        if tkk == 0.0:
            break
        V.append(v)
        z = E(cg_weighted_laplacian(w2, grad_T(Lw[None] * v), n_inner))
        Z.append(z)
        q = A(z)
        for i in range(k + 1):
            M[i, k] = _dot(q, U[i])
            q = q - M[i, k] * U[i]
        q, M[k + 1, k] = _normalise(q)
        U.append(q)
        y, lk, res = projected_tikhonov(M[: k + 2, : k + 1], beta1, rule, lam, noise_level)
        hist["res"].append(res)
        hist["lam"].append(lk)
        x = x0.copy()
        for i, yi in enumerate(y):
            x = x + yi * Z[i]
        if M[k + 1, k] == 0.0:
            break
    kk = len(Z)
    hist.update(res=np.asarray(hist["res"]), lam=np.asarray(hist["lam"]), U=U, V=V, Z=Z,
                M=M[: kk + 1, :kk], x0=x0)
    return x, hist
