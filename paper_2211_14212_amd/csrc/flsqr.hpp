// Internal declarations of the hybrid fLSQR-TV kernels (paper Sec. 2.3.2).
#pragma once

#include "krylov.hpp"

namespace kct {

// Scalar slots of fLSQR-TV and its inner CG (after the shared ones).
enum FlsqrScalar : int {
    S_FL_C0 = 36, // x0 = S_FL_C0 * 1, the best constant
    S_FL_CA,      // a^T a, a = A 1
    S_FL_E,       // coefficient of the current E / E^T correction
    S_FL_TKK,     // norm of the newest gradient-space vector before normalising
    S_CG_GAMMA,   // inner CG: ||r||^2
    S_CG_ALPHA,
    S_CG_BETA,
    S_CG_MU,      // mean of r, removed before the next direction
};
static_assert(S_CG_MU < S_COUNT, "scalar block too small");

int fl_groups(int64_t n);

// The inner CG runs in FP64 (vectors and stencil arithmetic).
// q = D^T (L^2 D p); partial sums of p.q.
kct_status fl_lap(const Plan &p, const double *pv, const float *Lw, double *q, double *parts, hipStream_t st);
// t += alpha p, r -= alpha q; partial sums of r and r^2.
kct_status fl_cg_update(double *t, double *r, const double *pv, const double *q, int64_t n, const double *S,
                        double *psum, double *psq, hipStream_t st);
// With rhs (FP32): r = rhs - mu, p = r, t = 0.  Without: r -= mu, p = r + beta p.
kct_status fl_cg_dir(double *r, double *pv, double *t, const float *rhs, int64_t n, const double *S, hipStream_t st);
// out = in rounded to FP32.
kct_status fl_to_f32(float *out, const double *in, int64_t n, hipStream_t st);
// out = D^T (L v3) for a gradient-space v3 (planar); partial sums of out and out^2.
kct_status fl_dtl(const Plan &p, const float *v3, const float *Lw, float *out, double *psum, double *psq,
                  hipStream_t st);
// Partial sums of v.
kct_status fl_sum(const float *v, int64_t n, double *parts, hipStream_t st);
// r -= S[ci] g; partial sums of r and r^2.
kct_status fl_axpy_sum(float *r, const float *g, int64_t n, const double *S, int ci, double *psum, double *psq,
                       hipStream_t st);
// out = in - S[ci].
kct_status fl_shift(float *out, const float *in, int64_t n, const double *S, int ci, hipStream_t st);
// out = S[ci].
kct_status fl_fill_s(float *out, int64_t n, const double *S, int ci, hipStream_t st);
// out = b + S[S_P0] a; partial sums of out^2.
kct_status fl_bbar(float *out, const float *b, const float *a, int64_t n, const double *S, double *parts,
                   hipStream_t st);
// x = S[S_FL_C0] + sum_{i < S[S_KGK]} coef_i Z_i.
kct_status fl_combine(float *x, const float *Z, int64_t n, const double *coef, const double *S, hipStream_t st);

kct_status fl_sc_init(double *S, Reduced ca, Reduced ab, int n_iter, double lam, hipStream_t st);
kct_status fl_sc_beta1(double *S, Reduced b2, hipStream_t st);
kct_status fl_sc_ecoef(double *S, Reduced dot, int ci, hipStream_t st);
kct_status fl_sc_cg_init(double *S, Reduced sum, Reduced sq, int64_t n, hipStream_t st);
kct_status fl_sc_cg_alpha(double *S, Reduced pq, hipStream_t st);
kct_status fl_sc_cg_beta(double *S, Reduced sum, Reduced sq, int64_t n, hipStream_t st);
kct_status fl_sc_vnorm(double *S, Reduced v2, hipStream_t st);
kct_status fl_sc_hist(double *S, const double *M, int k, int ldm, double *hist, hipStream_t st);

} // namespace kct
