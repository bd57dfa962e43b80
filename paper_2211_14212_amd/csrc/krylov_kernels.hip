// Vector and scalar kernels of the Krylov solvers (CGLS, LSQR, LSMR, hybrid
// LSQR), gfx950.
//
// Vector kernels stream volume- or projection-sized arrays (HBM-bound), apply
// one fused update per solver step and write one FP64 partial sum per
// workgroup.  Scalar kernels run as a single workgroup: they reduce the
// partial sums in a fixed order (so every run is bitwise identical), advance
// the method's FP64 recurrences, write one history row and leave the
// coefficients the next vector kernels read.  Nothing goes back to the host.
//
// Vectors the projectors read and write (CGLS r, q, p, s; GK u, v) are kept
// unnormalised in the Golub-Kahan methods: U holds beta_k u_k and V holds
// alpha_k v_k, and the 1/beta, 1/alpha factors travel as kernel coefficients.

#include "krylov.hpp"

namespace kct {

namespace {

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic sum over a 256-thread workgroup; the result is valid on thread 0.
__device__ inline double block_sum(double v)
{
    __shared__ double red[4];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// Sum of parts[0..n) by one workgroup, strided per thread in a fixed order.
__device__ inline double reduce_parts(const double *parts, int64_t n)
{
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += parts[e];
    return block_sum(s);
}

__global__ __launch_bounds__(256) void k_reduce_stage1(const double *__restrict__ parts, int64_t n,
                                                       double *__restrict__ out)
{
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * chunk, hi = min(n, lo + chunk);
    double s = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) s += parts[e];
    s = block_sum(s);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <typename T> __global__ __launch_bounds__(256) void k_fill(T *out, int64_t n, float v)
{
    const T val = from_f32<T>(v);
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) out[e] = val;
}

// out = c * in (c = scal[ci] if ci >= 0 else 1), partial sums of out^2.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_scale(const TI *__restrict__ in, TO *__restrict__ out, int64_t n,
                                               const double *scal, int ci, double *parts)
{
    const double c = ci >= 0 ? scal[ci] : 1.0;
    double s = 0.0;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const TO v = from_f32<TO>(float(c * double(to_f32(in[e]))));
        out[e] = v;
        const double f = to_f32(v);
        s += f * f;
    }
    if (parts) {
        s = block_sum(s);
        if (threadIdx.x == 0) parts[blockIdx.x] = s;
    }
}

// Projection-space update r = r + scal[P0] * q, partial sums of r^2.
template <typename T>
__global__ __launch_bounds__(256) void k_axpy_proj(T *__restrict__ r, const T *__restrict__ q, int64_t n,
                                                   const double *scal, double *parts)
{
    const double c = scal[S_P0];
    double s = 0.0;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const double re = to_f32(r[e]);
        const T v = from_f32<T>(float(c != 0.0 ? re + c * double(to_f32(q[e])) : re));
        r[e] = v;
        const double f = to_f32(v);
        s += f * f;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

// CGLS volume update: x += V0 p; p = V1 s + V2 p; partial sums of p^2.
template <typename T>
__global__ __launch_bounds__(256) void k_cgls_vol(float *__restrict__ x, T *__restrict__ p, const T *__restrict__ s,
                                                  int64_t n, const double *scal, double *parts)
{
    const double a = scal[S_V0], b1 = scal[S_V1], b2 = scal[S_V2];
    double acc = 0.0;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const double pe = to_f32(p[e]);
        if (a != 0.0) x[e] = float(double(x[e]) + a * pe);
        const double se = b1 != 0.0 ? b1 * double(to_f32(s[e])) : 0.0;
        const T pn = from_f32<T>(float(se + b2 * pe));
        p[e] = pn;
        const double f = to_f32(pn);
        acc += f * f;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

// LSQR volume update: x += V0 w; w = V1 V + V2 w.
template <typename T>
__global__ __launch_bounds__(256) void k_lsqr_vol(float *__restrict__ x, float *__restrict__ w,
                                                  const T *__restrict__ V, int64_t n, const double *scal)
{
    const double a = scal[S_V0], b1 = scal[S_V1], b2 = scal[S_V2];
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const double we = w[e];
        if (a != 0.0) x[e] = float(double(x[e]) + a * we);
        w[e] = float((b1 != 0.0 ? b1 * double(to_f32(V[e])) : 0.0) + b2 * we);
    }
}

// LSMR volume update: hbar = h + V0 hbar; x += V1 hbar; h = V2 V + V3 h.
template <typename T>
__global__ __launch_bounds__(256) void k_lsmr_vol(float *__restrict__ x, float *__restrict__ h,
                                                  float *__restrict__ hbar, const T *__restrict__ V, int64_t n,
                                                  const double *scal)
{
    const double c0 = scal[S_V0], c1 = scal[S_V1], c2 = scal[S_V2], c3 = scal[S_V3];
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const double he = h[e];
        const double hb = he + (c0 != 0.0 ? c0 * double(hbar[e]) : 0.0);
        hbar[e] = float(hb);
        if (c1 != 0.0) x[e] = float(double(x[e]) + c1 * double(float(hb)));
        h[e] = float((c2 != 0.0 ? c2 * double(to_f32(V[e])) : 0.0) + c3 * he);
    }
}

// Hybrid LSQR: x = sum_i coef[i] * basis[i], basis stored slot-major.
template <typename T>
__global__ __launch_bounds__(256) void k_combine(float *__restrict__ x, const T *__restrict__ basis, int64_t n,
                                                 const double *__restrict__ coef, const double *scal)
{
    const int k = int(scal[S_KGK]);
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += coef[i] * double(to_f32(basis[int64_t(i) * n + e]));
        x[e] = float(s);
    }
}

// ---------------------------------------------------------------------------
// Scalar kernels: one workgroup of 256 threads; thread 0 runs the recurrence.
// ---------------------------------------------------------------------------
__device__ inline void write_hist(double *hist, double *S, double res, double a, double b)
{
    if (hist) {
        const int64_t row = int64_t(S[S_HROW]);
        if (row < int64_t(S[S_ITER])) {
            double *h = hist + row * KCT_HIST_COLS;
            h[0] = res;
            h[1] = a;
            h[2] = b;
            h[3] = hist_code(S);
            h[4] = S[S_HLAM];
        }
    }
    S[S_HROW] += 1.0;
}

__device__ inline bool finite(double v) { return v == v && v - v == 0.0; }

// CGLS start: gamma = ||s||^2 with s = p = A^T b (minus lam^2 x0 = 0).
__global__ __launch_bounds__(256) void k_sc_cgls_init(double *S, const double *pa, int64_t na, double lam,
                                                      int n_iter)
{
    const double g = reduce_parts(pa, na);
    if (threadIdx.x != 0) return;
    S[S_LAMBDA] = lam;
    S[S_HLAM] = lam;
    S[S_PREV_EXPL] = -1.0;
    S[S_GAMMA] = g;
    S[S_PNORM2] = g;
    S[S_ITER] = n_iter;
    S[S_HROW] = 0.0;
    S[S_DONE] = !finite(g) ? 2.0 : (g == 0.0 ? 1.0 : 0.0);
    S[S_LAST] = 0.0;
}

// CGLS: delta = ||q||^2 + lam^2 ||p||^2, alpha = gamma / delta.
__global__ __launch_bounds__(256) void k_sc_cgls_alpha(double *S, const double *pq, int64_t nq,
                                                       const double *pp, int64_t np)
{
    const double q2 = reduce_parts(pq, nq);
    const double lam = S[S_LAMBDA];
    const double p2 = (lam != 0.0 && pp) ? reduce_parts(pp, np) : S[S_PNORM2];
    if (threadIdx.x != 0) return;
    double alpha = 0.0;
    if (S[S_DONE] == 0.0) {
        const double delta = q2 + lam * lam * p2;
        if (delta > 0.0 && finite(delta)) alpha = S[S_GAMMA] / delta;
        else S[S_DONE] = finite(delta) ? 1.0 : 2.0;
        S[S_DELTA] = delta;
    }
    S[S_ALPHA] = alpha;
    S[S_P0] = -alpha;                // r += P0 q
    S[S_B0] = 1.0;                   // s = A^T r - lam^2 (x + alpha p)
    S[S_B1] = 0.0;
    S[S_B2] = -lam * lam;
    S[S_B3] = -lam * lam * alpha;
}

// CGLS: gamma' = ||s||^2, beta = gamma'/gamma; history ||r||, alpha, beta.
__global__ __launch_bounds__(256) void k_sc_cgls_beta(double *S, const double *ps, int64_t ns,
                                                      const double *pr, int64_t nr, double *hist)
{
    const double s2 = reduce_parts(ps, ns);
    const double r2 = reduce_parts(pr, nr);
    if (threadIdx.x != 0) return;
    const bool was_done = S[S_ALPHA] == 0.0;
    double beta = 0.0;
    if (!was_done) {
        beta = s2 / S[S_GAMMA];
        S[S_GAMMA] = s2;
        if (!finite(s2)) S[S_DONE] = 2.0;
        else if (!(s2 > 0.0)) S[S_DONE] = 1.0;
        S[S_RES] = sqrt(r2);
    }
    S[S_BETA] = beta;
    S[S_V0] = S[S_ALPHA];           // x += alpha p
    S[S_V1] = was_done ? 0.0 : 1.0; // p = s + beta p
    S[S_V2] = was_done ? 1.0 : beta;
    write_hist(hist, S, S[S_RES], S[S_ALPHA], beta);
}

// Golub-Kahan start, part 1: beta_1 = ||b||, back projector scales by 1/beta_1.
__global__ __launch_bounds__(256) void k_sc_gk_init1(double *S, const double *pu, int64_t nu, double lam,
                                                     int n_iter)
{
    const double b2 = reduce_parts(pu, nu);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(b2);
    S[S_LAMBDA] = lam;
    S[S_HLAM] = lam;
    S[S_PREV_EXPL] = -1.0;
    S[S_ITER] = n_iter;
    S[S_HROW] = 0.0;
    S[S_KGK] = 0.0;
    S[S_BETA] = beta;
    S[S_DONE] = !finite(beta) ? 2.0 : (beta > 0.0 ? 0.0 : 1.0);
    S[S_LAST] = 0.0;
    S[S_B0] = S[S_DONE] == 0.0 ? 1.0 / beta : 0.0;
    S[S_B1] = S[S_B2] = S[S_B3] = 0.0;
}

// Golub-Kahan start, part 2: alpha_1 = ||A^T u_1||; LSQR/LSMR initial scalars.
__global__ __launch_bounds__(256) void k_sc_gk_init2(double *S, const double *pv, int64_t nv, double *gk)
{
    const double a2 = reduce_parts(pv, nv);
    if (threadIdx.x != 0) return;
    const double alpha = S[S_DONE] == 0.0 ? sqrt(a2) : 0.0;
    const double beta = S[S_BETA];
    if (!finite(alpha)) S[S_DONE] = 2.0;
    else if (!(alpha > 0.0) && S[S_DONE] == 0.0) S[S_DONE] = 1.0;
    S[S_ALPHA] = alpha;
    // LSQR
    S[S_PHIBAR] = beta;
    S[S_RHOBAR] = alpha;
    S[S_PSISQ] = 0.0;
    // LSMR
    S[S_ALPHABAR] = alpha;
    S[S_ZETABAR] = alpha * beta;
    S[S_RHO_OLD] = 1.0;
    S[S_RHOBAR_OLD] = 1.0;
    S[S_CBAR] = 1.0;
    S[S_SBAR] = 0.0;
    const bool ok = S[S_DONE] == 0.0;
    S[S_V0] = ok ? 1.0 / alpha : 0.0; // w (or h) = V / alpha_1
    S[S_F0] = ok ? 1.0 / alpha : 0.0; // U = (1/alpha) A V - (alpha/beta) U
    S[S_F1] = ok ? -alpha / beta : 0.0;
    if (gk) {
        gk[0] = beta;  // beta_1
        gk[1] = alpha; // alpha_1
    }
}

// Golub-Kahan: beta_{k+1} = ||U||; back projector coefficients.
__global__ __launch_bounds__(256) void k_sc_gk_beta(double *S, const double *pu, int64_t nu)
{
    const double b2 = reduce_parts(pu, nu);
    if (threadIdx.x != 0) return;
    if (S[S_DONE] != 0.0) return;
    const double beta = sqrt(b2);
    const double alpha = S[S_ALPHA];
    S[S_BETA] = beta;
    S[S_LAST] = (beta > 0.0 && finite(beta)) ? 0.0 : (finite(beta) ? 1.0 : 2.0);
    if (!finite(beta)) S[S_BETA] = 0.0;
    const bool ok = S[S_LAST] == 0.0;
    S[S_B0] = ok ? 1.0 / beta : 0.0; // V = (1/beta) A^T U - (beta/alpha) V
    S[S_B1] = ok ? -beta / alpha : 0.0;
    S[S_B2] = S[S_B3] = 0.0;
}

// LSQR (damped): alpha_{k+1}, the two plane rotations, update coefficients.
__global__ __launch_bounds__(256) void k_sc_lsqr_alpha(double *S, const double *pv, int64_t nv, double *hist,
                                                       double *gk)
{
    const double a2 = reduce_parts(pv, nv);
    if (threadIdx.x != 0) return;
    if (S[S_DONE] != 0.0) {
        S[S_V0] = 0.0; // x unchanged
        S[S_V1] = 0.0;
        S[S_V2] = 1.0;
        write_hist(hist, S, sqrt(S[S_PHIBAR] * S[S_PHIBAR] + S[S_PSISQ]), S[S_ALPHA], S[S_BETA]);
        return;
    }
    const double lam = S[S_LAMBDA];
    const bool last = S[S_LAST] != 0.0;
    double alpha = last ? 0.0 : sqrt(a2);
    const bool bad = !finite(alpha) || S[S_LAST] == 2.0;
    if (!finite(alpha)) alpha = 0.0;
    const double beta = S[S_BETA];
    // Fold the damping row into rhobar.
    const double rhobar = S[S_RHOBAR];
    const double rhohat = sqrt(rhobar * rhobar + lam * lam);
    const double c1 = rhobar / rhohat, s1 = lam / rhohat;
    const double psi = s1 * S[S_PHIBAR];
    double phibar = c1 * S[S_PHIBAR];
    S[S_PSISQ] += psi * psi;
    // Eliminate beta_{k+1}.
    const double rho = sqrt(rhohat * rhohat + beta * beta);
    const double c = rhohat / rho, s = beta / rho;
    const double theta = s * alpha;
    S[S_RHOBAR] = -c * alpha;
    const double phi = c * phibar;
    phibar = s * phibar;
    S[S_PHIBAR] = phibar;
    S[S_V0] = phi / rho;                      // x += (phi/rho) w
    S[S_V1] = alpha > 0.0 ? 1.0 / alpha : 0.0; // w = V/alpha - (theta/rho) w
    S[S_V2] = -theta / rho;
    S[S_F0] = alpha > 0.0 ? 1.0 / alpha : 0.0;
    S[S_F1] = alpha > 0.0 ? -alpha / beta : 0.0;
    if (gk) {
        const int k = int(S[S_KGK]);
        gk[2 * k + 2] = beta;  // beta_{k+2}
        gk[2 * k + 3] = alpha; // alpha_{k+2}
    }
    S[S_KGK] += 1.0;
    S[S_ALPHA] = alpha;
    if (last || alpha == 0.0) S[S_DONE] = bad ? 2.0 : 1.0;
    write_hist(hist, S, sqrt(phibar * phibar + S[S_PSISQ]), alpha, beta);
}

// LSMR (damped): alpha_{k+1} and the rotations of Fong and Saunders.
__global__ __launch_bounds__(256) void k_sc_lsmr_alpha(double *S, const double *pv, int64_t nv, double *hist)
{
    const double a2 = reduce_parts(pv, nv);
    if (threadIdx.x != 0) return;
    if (S[S_DONE] != 0.0) {
        S[S_V0] = 0.0;
        S[S_V1] = 0.0; // x unchanged
        S[S_V2] = 0.0;
        S[S_V3] = 1.0;
        write_hist(hist, S, fabs(S[S_ZETABAR]), S[S_ALPHA], S[S_BETA]);
        return;
    }
    const double lam = S[S_LAMBDA];
    const bool last = S[S_LAST] != 0.0;
    double alpha = last ? 0.0 : sqrt(a2);
    const bool bad = !finite(alpha) || S[S_LAST] == 2.0;
    if (!finite(alpha)) alpha = 0.0;
    const double beta = S[S_BETA];
    const double alphabar = S[S_ALPHABAR];
    const double alphahat = sqrt(alphabar * alphabar + lam * lam);
    const double rho = sqrt(alphahat * alphahat + beta * beta);
    const double c = alphahat / rho, s = beta / rho;
    const double theta_next = s * alpha;
    S[S_ALPHABAR] = c * alpha;
    const double sbar_old = S[S_SBAR], cbar_old = S[S_CBAR];
    const double thetabar = sbar_old * rho;
    const double rhobar = sqrt((cbar_old * rho) * (cbar_old * rho) + theta_next * theta_next);
    const double cbar = cbar_old * rho / rhobar;
    const double sbar = theta_next / rhobar;
    const double zeta = cbar * S[S_ZETABAR];
    const double zetabar = -sbar * S[S_ZETABAR];
    S[S_V0] = -thetabar * rho / (S[S_RHO_OLD] * S[S_RHOBAR_OLD]); // hbar = h + V0 hbar
    S[S_V1] = zeta / (rho * rhobar);                            // x += V1 hbar
    S[S_V2] = alpha > 0.0 ? 1.0 / alpha : 0.0;                  // h = V/alpha - (theta/rho) h
    S[S_V3] = -theta_next / rho;
    S[S_F0] = alpha > 0.0 ? 1.0 / alpha : 0.0;
    S[S_F1] = alpha > 0.0 ? -alpha / beta : 0.0;
    S[S_CBAR] = cbar;
    S[S_SBAR] = sbar;
    S[S_ZETABAR] = zetabar;
    S[S_RHO_OLD] = rho;
    S[S_RHOBAR_OLD] = rhobar;
    S[S_ALPHA] = alpha;
    if (last || alpha == 0.0) S[S_DONE] = bad ? 2.0 : 1.0;
    write_hist(hist, S, fabs(zetabar), alpha, beta);
}

// Hybrid LSQR final step: y = argmin ||[B_k; lam I] y - [beta_1 e_1; 0]||
// by Householder QR in FP64 (thread 0), then coef[i] = y_i / alpha_i so that
// x = sum_i coef[i] * (stored unnormalised basis vector i).
__global__ __launch_bounds__(64) void k_hybrid_solve(double *S, const double *gk, double *work, double *coef)
{
    if (threadIdx.x != 0) return;
    const int k = int(S[S_KGK]);
    const double lam = S[S_LAMBDA];
    const int m = 2 * k + 1;
    double *M = work;            // m x k, column-major
    double *rhs = work + m * k;  // m
    for (int e = 0; e < m * k; ++e) M[e] = 0.0;
    for (int e = 0; e < m; ++e) rhs[e] = 0.0;
    rhs[0] = gk[0];
    for (int c = 0; c < k; ++c) {
        M[c * m + c] = gk[2 * c + 1];     // alpha_{c+1}
        M[c * m + c + 1] = gk[2 * c + 2]; // beta_{c+2}
        M[c * m + k + 1 + c] = lam;
    }
    for (int c = 0; c < k; ++c) {
        double nrm = 0.0;
        for (int r = c; r < m; ++r) nrm += M[c * m + r] * M[c * m + r];
        nrm = sqrt(nrm);
        if (nrm == 0.0) continue;
        const double alpha = M[c * m + c] > 0.0 ? -nrm : nrm;
        double v0 = M[c * m + c] - alpha;
        // Householder vector v = (v0, M[c+1..m-1, c]); H = I - 2 v v^T / (v^T v).
        double vtv = v0 * v0;
        for (int r = c + 1; r < m; ++r) vtv += M[c * m + r] * M[c * m + r];
        for (int cc = c + 1; cc < k; ++cc) {
            double d = v0 * M[cc * m + c];
            for (int r = c + 1; r < m; ++r) d += M[c * m + r] * M[cc * m + r];
            const double f = 2.0 * d / vtv;
            M[cc * m + c] -= f * v0;
            for (int r = c + 1; r < m; ++r) M[cc * m + r] -= f * M[c * m + r];
        }
        double d = v0 * rhs[c];
        for (int r = c + 1; r < m; ++r) d += M[c * m + r] * rhs[r];
        const double f = 2.0 * d / vtv;
        rhs[c] -= f * v0;
        for (int r = c + 1; r < m; ++r) rhs[r] -= f * M[c * m + r];
        M[c * m + c] = alpha;
    }
    for (int c = k - 1; c >= 0; --c) {
        double v = rhs[c];
        for (int cc = c + 1; cc < k; ++cc) v -= M[cc * m + c] * coef[cc];
        coef[c] = M[c * m + c] != 0.0 ? v / M[c * m + c] : 0.0;
    }
    for (int c = 0; c < k; ++c) coef[c] /= gk[2 * c + 1];
}

// ---------------------------------------------------------------------------
// Explicit residual and stop rule: after each iteration ||b - A x_k|| comes
// from the forward projector's partial sums into history column 0.  With the
// stop rule, x_prev = x before each iteration while the run is live, and when
// the residual exceeds the previous one the run is done (3) and x is put back
// to x_prev on this and every later iteration (idempotent: x_prev no longer
// moves).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_save_x(const float *__restrict__ x, float *__restrict__ xp, int64_t n,
                                                const double *__restrict__ S)
{
    if (S[S_DONE] != 0.0) return;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) xp[e] = x[e];
}

__global__ __launch_bounds__(256) void k_restore_x(float *__restrict__ x, const float *__restrict__ xp, int64_t n,
                                                   const double *__restrict__ S)
{
    if (S[S_DONE] != 3.0) return;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) x[e] = xp[e];
}

__global__ __launch_bounds__(256) void k_sc_explicit(double *S, const double *p, int64_t n, double *hist,
                                                    int stop)
{
    const double r2 = reduce_parts(p, n);
    if (threadIdx.x != 0) return;
    const double r = sqrt(r2);
    if (S[S_DONE] == 0.0) {
        if (!finite(r)) S[S_DONE] = 2.0;
        else if (stop && S[S_PREV_EXPL] >= 0.0 && r > S[S_PREV_EXPL]) S[S_DONE] = 3.0;
        else S[S_PREV_EXPL] = r;
    }
    if (hist) {
        const int64_t row = int64_t(S[S_HROW]) - 1;
        if (row >= 0 && row < int64_t(S[S_ITER])) {
            hist[row * KCT_HIST_COLS + 0] = r;
            hist[row * KCT_HIST_COLS + 3] = hist_code(S);
        }
    }
}

// ---------------------------------------------------------------------------
// Hybrid LSQR with lambda_k chosen at every iteration (GCV or discrepancy
// principle on the projected problem), and the projected solve of hybrid
// fLSQR-TV.  One workgroup:
//   1. B_k ((k+1) x k: lower bidiagonal from the stored alpha, beta, or the
//      upper Hessenberg M_k of the flexible process) is copied to W, and Q = I;
//   2. one-sided Jacobi: pairs of columns of W are rotated until they are
//      orthogonal (round-robin pair order, k/2 pairs per round, one thread per
//      pair), the same rotations accumulate in Q; then sigma_i = ||W_i||,
//      P_i = W_i / sigma_i, B_k = P diag(sigma) Q^T;
//   3. c_i = beta_1 P_i[0] for i < k, and c_k = beta_1 n_0 / ||n|| with n the
//      null vector of B_k^T (n_0 = 1, n_{j+1} = -sum_{i<=j} n_i B[i, j] /
//      B[j+1, j], for the bidiagonal -alpha_{j+1} n_j / beta_{j+2}): the part
//      of beta_1 e_1 outside the range of B_k;
//   4. lambda_k by the rule (the same search as the oracle's);
//   5. y = Q diag(sigma / (sigma^2 + lambda^2)) c; coef_i = y_i / alpha_i for
//      the unnormalised GK basis, y_i for fLSQR-TV; history row k gets the
//      projected Tikhonov residual and lambda_k.
// ---------------------------------------------------------------------------
namespace hyb {

constexpr int GRID = 81;       // log10 lambda grid: sigma_max * 10^[-7, 1]
constexpr int GOLDEN = 60;     // golden-section steps
constexpr int BISECT = 64;     // bisection steps on log10 lambda, sigma_max * 10^[-12, 8]
constexpr int SWEEPS = 60;     // Jacobi sweep limit
constexpr double EPS = 2.220446049250313e-16;

__device__ inline double res2(const double *sig, const double *c, int k, double lam)
{
    double r = c[k] * c[k];
    for (int i = 0; i < k; ++i) {
        const double s2 = sig[i] * sig[i];
        const double f = s2 > 0.0 ? s2 / (s2 + lam * lam) : 0.0;
        const double t = (1.0 - f) * c[i];
        r += t * t;
    }
    return r;
}

__device__ inline double gcv(const double *sig, const double *c, int k, double lam)
{
    double tr = 1.0;
    for (int i = 0; i < k; ++i) {
        const double s2 = sig[i] * sig[i];
        tr += 1.0 - (s2 > 0.0 ? s2 / (s2 + lam * lam) : 0.0);
    }
    return res2(sig, c, k, lam) / (tr * tr);
}

} // namespace hyb

// DENSE: src is M_k column-major with leading dimension ldm and beta_1 is
// S[S_BETA]; otherwise src is the interleaved [beta_1, alpha_1, beta_2, ...].
template <bool DENSE>
__device__ void hybrid_choose_body(double *S, const double *src, int ldm, double *work, double *coef, double *hist,
                                   int rule, double noise_level)
{
    using namespace hyb;
    __shared__ int rotated;
    __shared__ double grid_g[GRID];
    __shared__ double sh_lam, sh_smax;
    const int tid = threadIdx.x;
    if (S[S_DONE] == 2.0) return;
    const int k = int(S[S_KGK]);
    if (k <= 0) return;
    const int m = k + 1;
    double *W = work;         // m x k, column-major
    double *Q = W + m * k;    // k x k, column-major
    double *sig = Q + k * k;  // k
    double *c = sig + k;      // k + 1
    double *y = c + k + 1;    // k
    const double beta1 = DENSE ? S[S_BETA] : src[0];

    for (int e = tid; e < k * k; e += 256) Q[e] = (e % (k + 1) == 0) ? 1.0 : 0.0;
    if constexpr (DENSE) {
        for (int e = tid; e < m * k; e += 256) {
            const int j = e / m, i = e - j * m;
            W[e] = i <= j + 1 ? src[int64_t(j) * ldm + i] : 0.0;
        }
        __syncthreads();
    } else {
        for (int e = tid; e < m * k; e += 256) W[e] = 0.0;
        __syncthreads();
        for (int j = tid; j < k; j += 256) {
            W[j * m + j] = src[2 * j + 1];     // alpha_{j+1}
            W[j * m + j + 1] = src[2 * j + 2]; // beta_{j+2}
        }
    }
    __syncthreads();

    // Round-robin order over n2 (even) slots; slot k is empty when k is odd.
    const int n2 = k + (k & 1);
    // Rotate while |w_p . w_q| > (k+1) eps ||w_p|| ||w_q||, the rounding level
    // of the dot products.
    const double tol = double(m) * EPS;
    for (int sweep = 0; sweep < SWEEPS && n2 > 1; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < n2 - 1; ++r) {
            for (int pi = tid; pi < n2 / 2; pi += 256) {
                int p, q;
                if (pi == 0) {
                    p = r;
                    q = n2 - 1;
                } else {
                    p = (r + pi) % (n2 - 1);
                    q = (r - pi + (n2 - 1)) % (n2 - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                if (q >= k) continue;
                double *wp = W + p * m, *wq = W + q * m;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = 0; i < m; ++i) {
                    a += wp[i] * wp[i];
                    b += wq[i] * wq[i];
                    g += wp[i] * wq[i];
                }
                if (g != 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
                    const double zeta = (b - a) / (2.0 * g);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                    for (int i = 0; i < m; ++i) {
                        const double u = wp[i], v = wq[i];
                        wp[i] = cs * u - sn * v;
                        wq[i] = sn * u + cs * v;
                    }
                    double *qp = Q + p * k, *qq = Q + q * k;
                    for (int i = 0; i < k; ++i) {
                        const double u = qp[i], v = qq[i];
                        qp[i] = cs * u - sn * v;
                        qq[i] = sn * u + cs * v;
                    }
                    rotated = 1;
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }

    for (int j = tid; j < k; j += 256) {
        double s2 = 0.0;
        for (int i = 0; i < m; ++i) s2 += W[j * m + i] * W[j * m + i];
        const double sg = sqrt(s2);
        sig[j] = sg;
        c[j] = sg > 0.0 ? beta1 * W[j * m] / sg : 0.0;
    }
    if (tid == 0) {
        // c_k from the null vector of B_k^T, rescaled to stay in range.
        if constexpr (DENSE) {
            double *nv = y + k; // k + 1 entries
            double ssq = 1.0;
            bool zero = false;
            nv[0] = 1.0;
            for (int j = 0; j < k; ++j) {
                const double *col = src + int64_t(j) * ldm;
                if (col[j + 1] == 0.0) {
                    zero = true;
                    break;
                }
                double t = 0.0;
                for (int i = 0; i <= j; ++i) t += nv[i] * col[i];
                nv[j + 1] = -t / col[j + 1];
                ssq += nv[j + 1] * nv[j + 1];
                if (fabs(nv[j + 1]) > 1e100) {
                    for (int i = 0; i <= j + 1; ++i) nv[i] *= 1e-100;
                    ssq *= 1e-200;
                }
            }
            c[k] = zero ? 0.0 : beta1 * nv[0] / sqrt(ssq);
        } else {
            double n0 = 1.0, cur = 1.0, ssq = 1.0;
            bool zero = false;
            for (int j = 0; j < k && !zero; ++j) {
                const double al = src[2 * j + 1], be = src[2 * j + 2];
                if (be == 0.0) {
                    zero = true;
                    break;
                }
                cur = -al * cur / be;
                ssq += cur * cur;
                if (fabs(cur) > 1e100) {
                    cur *= 1e-100;
                    ssq *= 1e-200;
                    n0 *= 1e-100;
                }
            }
            c[k] = zero ? 0.0 : beta1 * n0 / sqrt(ssq);
        }
    }
    __syncthreads();
    if (tid == 0) {
        double smax = 0.0;
        for (int j = 0; j < k; ++j) smax = fmax(smax, sig[j]);
        sh_smax = smax;
    }
    __syncthreads();
    const double smax = sh_smax;

    if (rule == KCT_LAMBDA_GCV) {
        const double L = log10(smax);
        if (smax > 0.0 && tid < GRID) grid_g[tid] = gcv(sig, c, k, pow(10.0, L - 7.0 + 8.0 * tid / (GRID - 1)));
        __syncthreads();
        if (tid == 0) {
            double lam = 0.0;
            if (smax > 0.0) {
                int j = 0;
                for (int t = 1; t < GRID; ++t)
                    if (grid_g[t] < grid_g[j]) j = t;
                const double gj0 = L - 7.0 + 8.0 * max(j - 1, 0) / (GRID - 1);
                const double gj1 = L - 7.0 + 8.0 * min(j + 1, GRID - 1) / (GRID - 1);
                double a = gj0, b = gj1;
                const double rr = (sqrt(5.0) - 1.0) / 2.0;
                double x1 = b - rr * (b - a), x2 = a + rr * (b - a);
                double f1 = gcv(sig, c, k, pow(10.0, x1)), f2 = gcv(sig, c, k, pow(10.0, x2));
                for (int it = 0; it < GOLDEN; ++it) {
                    if (f1 <= f2) {
                        b = x2;
                        x2 = x1;
                        f2 = f1;
                        x1 = b - rr * (b - a);
                        f1 = gcv(sig, c, k, pow(10.0, x1));
                    } else {
                        a = x1;
                        x1 = x2;
                        f1 = f2;
                        x2 = a + rr * (b - a);
                        f2 = gcv(sig, c, k, pow(10.0, x2));
                    }
                }
                lam = pow(10.0, 0.5 * (a + b));
            }
            sh_lam = lam;
        }
    } else if (tid == 0) {
        double lam = 0.0;
        if (rule == KCT_LAMBDA_DP && smax > 0.0) {
            const double target = (noise_level * beta1) * (noise_level * beta1);
            double call = 0.0;
            for (int j = 0; j <= k; ++j) call += c[j] * c[j];
            if (c[k] * c[k] >= target) {
                lam = 0.0;
            } else if (call <= target) {
                lam = HUGE_VAL;
            } else {
                const double L = log10(smax);
                double lo = L - 12.0, hi = L + 8.0;
                for (int it = 0; it < BISECT; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (res2(sig, c, k, pow(10.0, mid)) < target) lo = mid;
                    else hi = mid;
                }
                lam = pow(10.0, 0.5 * (lo + hi));
            }
        } else if (rule == KCT_LAMBDA_FIXED) {
            lam = S[S_LAMBDA];
        }
        sh_lam = lam;
    }
    __syncthreads();
    const double lam = sh_lam;
    const bool inf = !(lam < HUGE_VAL);

    for (int r = tid; r < k; r += 256) {
        double v = 0.0;
        if (!inf)
            for (int i = 0; i < k; ++i) {
                const double s2 = sig[i] * sig[i];
                const double gi = s2 > 0.0 ? sig[i] / (s2 + lam * lam) : 0.0;
                v += Q[i * k + r] * (gi * c[i]);
            }
        y[r] = v;
        coef[r] = DENSE ? v : v / src[2 * r + 1];
    }
    __syncthreads();
    if (tid == 0) {
        double res = beta1;
        if (!inf) {
            double yy = 0.0;
            for (int r = 0; r < k; ++r) yy += y[r] * y[r];
            res = sqrt(res2(sig, c, k, lam) + lam * lam * yy);
        }
        S[S_HLAM] = lam;
        if (hist) {
            const int64_t row = int64_t(S[S_HROW]) - 1;
            if (row >= 0 && row < int64_t(S[S_ITER])) {
                hist[row * KCT_HIST_COLS + 0] = res;
                hist[row * KCT_HIST_COLS + 4] = lam;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_hybrid_choose(double *S, const double *gk, double *work, double *coef,
                                                       double *hist, int rule, double noise_level)
{
    hybrid_choose_body<false>(S, gk, 0, work, coef, hist, rule, noise_level);
}

__global__ __launch_bounds__(256) void k_hybrid_choose_dense(double *S, const double *M, int ldm, double *work,
                                                             double *coef, double *hist, int rule, double noise_level)
{
    hybrid_choose_body<true>(S, M, ldm, work, coef, hist, rule, noise_level);
}

int vec_groups(int64_t n)
{
    const int64_t g = (n + 1023) / 1024;
    return int(std::max<int64_t>(1, std::min<int64_t>(g, VEC_GROUPS)));
}

} // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
#define KCT_DT_DISPATCH(dt, T, ...)                                                                                \
    switch (dt) {                                                                                                  \
    case KCT_F32: { using T = float; __VA_ARGS__; } break;                                                        \
    case KCT_BF16: { using T = bf16; __VA_ARGS__; } break;                                                        \
    case KCT_F16: { using T = _Float16; __VA_ARGS__; } break;                                                     \
    default: return fail(KCT_E_DTYPE, "unsupported storage type");                                               \
    }

Reduced reduce_for_scalar(const double *parts, int64_t n, double *stage, hipStream_t st)
{
    if (n <= 4096) return {parts, n};
    hipLaunchKernelGGL(k_reduce_stage1, dim3(256), dim3(256), 0, st, parts, n, stage);
    return {stage, 256};
}

kct_status vk_fill(void *out, int dt, int64_t n, float v, hipStream_t st)
{
    KCT_DT_DISPATCH(dt, T, hipLaunchKernelGGL(k_fill<T>, dim3(vec_groups(n)), dim3(256), 0, st,
                                              static_cast<T *>(out), n, v));
    return check_hip(hipGetLastError(), "fill");
}

kct_status vk_scale(const void *in, int dti, void *out, int dto, int64_t n, const double *scal, int ci,
                    double *parts, hipStream_t st)
{
    if (dti == KCT_F32) {
        KCT_DT_DISPATCH(dto, TO, hipLaunchKernelGGL((k_scale<float, TO>), dim3(vec_groups(n)), dim3(256), 0, st,
                                                    static_cast<const float *>(in), static_cast<TO *>(out), n, scal,
                                                    ci, parts));
    } else if (dto == KCT_F32) {
        KCT_DT_DISPATCH(dti, TI, hipLaunchKernelGGL((k_scale<TI, float>), dim3(vec_groups(n)), dim3(256), 0, st,
                                                    static_cast<const TI *>(in), static_cast<float *>(out), n, scal,
                                                    ci, parts));
    } else if (dti == dto) {
        KCT_DT_DISPATCH(dti, T, hipLaunchKernelGGL((k_scale<T, T>), dim3(vec_groups(n)), dim3(256), 0, st,
                                                   static_cast<const T *>(in), static_cast<T *>(out), n, scal, ci,
                                                   parts));
    } else {
        return fail(KCT_E_DTYPE, "unsupported conversion");
    }
    return check_hip(hipGetLastError(), "scale");
}

kct_status vk_axpy_proj(void *r, const void *q, int dt, int64_t n, const double *scal, double *parts,
                        hipStream_t st)
{
    KCT_DT_DISPATCH(dt, T, hipLaunchKernelGGL(k_axpy_proj<T>, dim3(vec_groups(n)), dim3(256), 0, st,
                                              static_cast<T *>(r), static_cast<const T *>(q), n, scal, parts));
    return check_hip(hipGetLastError(), "projection update");
}

kct_status vk_cgls_vol(float *x, void *p, const void *s, int dt, int64_t n, const double *scal, double *parts,
                       hipStream_t st)
{
    KCT_DT_DISPATCH(dt, T, hipLaunchKernelGGL(k_cgls_vol<T>, dim3(vec_groups(n)), dim3(256), 0, st, x,
                                              static_cast<T *>(p), static_cast<const T *>(s), n, scal, parts));
    return check_hip(hipGetLastError(), "cgls update");
}

kct_status vk_lsqr_vol(float *x, float *w, const void *V, int dt, int64_t n, const double *scal, hipStream_t st)
{
    KCT_DT_DISPATCH(dt, T, hipLaunchKernelGGL(k_lsqr_vol<T>, dim3(vec_groups(n)), dim3(256), 0, st, x, w,
                                              static_cast<const T *>(V), n, scal));
    return check_hip(hipGetLastError(), "lsqr update");
}

kct_status vk_lsmr_vol(float *x, float *h, float *hbar, const void *V, int dt, int64_t n, const double *scal,
                       hipStream_t st)
{
    KCT_DT_DISPATCH(dt, T, hipLaunchKernelGGL(k_lsmr_vol<T>, dim3(vec_groups(n)), dim3(256), 0, st, x, h, hbar,
                                              static_cast<const T *>(V), n, scal));
    return check_hip(hipGetLastError(), "lsmr update");
}

kct_status vk_combine(float *x, const void *basis, int dt, int64_t n, const double *coef, const double *scal,
                      hipStream_t st)
{
    KCT_DT_DISPATCH(dt, T, hipLaunchKernelGGL(k_combine<T>, dim3(vec_groups(n)), dim3(256), 0, st, x,
                                              static_cast<const T *>(basis), n, coef, scal));
    return check_hip(hipGetLastError(), "basis combination");
}

int vk_groups(int64_t n) { return vec_groups(n); }

#define SC1(...) hipLaunchKernelGGL(__VA_ARGS__)

kct_status sk_cgls_init(double *S, Reduced p, double lam, int n_iter, hipStream_t st)
{
    SC1(k_sc_cgls_init, dim3(1), dim3(256), 0, st, S, p.ptr, p.n, lam, n_iter);
    return check_hip(hipGetLastError(), "cgls init scalars");
}
kct_status sk_cgls_alpha(double *S, Reduced q, Reduced p, hipStream_t st)
{
    SC1(k_sc_cgls_alpha, dim3(1), dim3(256), 0, st, S, q.ptr, q.n, p.ptr, p.n);
    return check_hip(hipGetLastError(), "cgls alpha");
}
kct_status sk_cgls_beta(double *S, Reduced s, Reduced r, double *hist, hipStream_t st)
{
    SC1(k_sc_cgls_beta, dim3(1), dim3(256), 0, st, S, s.ptr, s.n, r.ptr, r.n, hist);
    return check_hip(hipGetLastError(), "cgls beta");
}
kct_status sk_gk_init1(double *S, Reduced u, double lam, int n_iter, hipStream_t st)
{
    SC1(k_sc_gk_init1, dim3(1), dim3(256), 0, st, S, u.ptr, u.n, lam, n_iter);
    return check_hip(hipGetLastError(), "gk init");
}
kct_status sk_gk_init2(double *S, Reduced v, double *gk, hipStream_t st)
{
    SC1(k_sc_gk_init2, dim3(1), dim3(256), 0, st, S, v.ptr, v.n, gk);
    return check_hip(hipGetLastError(), "gk init 2");
}
kct_status sk_gk_beta(double *S, Reduced u, hipStream_t st)
{
    SC1(k_sc_gk_beta, dim3(1), dim3(256), 0, st, S, u.ptr, u.n);
    return check_hip(hipGetLastError(), "gk beta");
}
kct_status sk_lsqr_alpha(double *S, Reduced v, double *hist, double *gk, hipStream_t st)
{
    SC1(k_sc_lsqr_alpha, dim3(1), dim3(256), 0, st, S, v.ptr, v.n, hist, gk);
    return check_hip(hipGetLastError(), "lsqr alpha");
}
kct_status sk_lsmr_alpha(double *S, Reduced v, double *hist, hipStream_t st)
{
    SC1(k_sc_lsmr_alpha, dim3(1), dim3(256), 0, st, S, v.ptr, v.n, hist);
    return check_hip(hipGetLastError(), "lsmr alpha");
}
kct_status sk_hybrid_solve(double *S, const double *gk, double *work, double *coef, hipStream_t st)
{
    SC1(k_hybrid_solve, dim3(1), dim3(64), 0, st, S, gk, work, coef);
    return check_hip(hipGetLastError(), "hybrid projected solve");
}
kct_status vk_save_x(const float *x, float *xp, int64_t n, const double *S, hipStream_t st)
{
    hipLaunchKernelGGL(k_save_x, dim3(vec_groups(n)), dim3(256), 0, st, x, xp, n, S);
    return check_hip(hipGetLastError(), "save x");
}
kct_status vk_restore_x(float *x, const float *xp, int64_t n, const double *S, hipStream_t st)
{
    hipLaunchKernelGGL(k_restore_x, dim3(vec_groups(n)), dim3(256), 0, st, x, xp, n, S);
    return check_hip(hipGetLastError(), "restore x");
}
kct_status sk_explicit(double *S, Reduced r, double *hist, bool stop, hipStream_t st)
{
    SC1(k_sc_explicit, dim3(1), dim3(256), 0, st, S, r.ptr, r.n, hist, stop ? 1 : 0);
    return check_hip(hipGetLastError(), "explicit residual");
}
kct_status sk_hybrid_choose(double *S, const double *gk, double *work, double *coef, double *hist, int rule,
                            double noise_level, hipStream_t st)
{
    SC1(k_hybrid_choose, dim3(1), dim3(256), 0, st, S, gk, work, coef, hist, rule, noise_level);
    return check_hip(hipGetLastError(), "hybrid parameter choice");
}
kct_status sk_hybrid_choose_dense(double *S, const double *M, int ldm, double *work, double *coef, double *hist,
                                  int rule, double noise_level, hipStream_t st)
{
    SC1(k_hybrid_choose_dense, dim3(1), dim3(256), 0, st, S, M, ldm, work, coef, hist, rule, noise_level);
    return check_hip(hipGetLastError(), "projected Tikhonov solve");
}

} // namespace kct
