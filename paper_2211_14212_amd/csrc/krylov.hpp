// Internal declarations of the Krylov vector and scalar kernels.
#pragma once

#include <algorithm>

#include "kct_internal.hpp"

namespace kct {

constexpr int VEC_GROUPS = 2048; // workgroups of the streaming vector kernels

// A partial-sum array ready for a scalar kernel (at most a few thousand entries).
struct Reduced {
    const double *ptr;
    int64_t n;
};

// Shrink `n` per-workgroup partial sums to 256 (in `stage`) when there are many.
Reduced reduce_for_scalar(const double *parts, int64_t n, double *stage, hipStream_t st);

int vk_groups(int64_t n);
kct_status vk_fill(void *out, int dt, int64_t n, float v, hipStream_t st);
kct_status vk_scale(const void *in, int dti, void *out, int dto, int64_t n, const double *scal, int ci,
                    double *parts, hipStream_t st);
kct_status vk_axpy_proj(void *r, const void *q, int dt, int64_t n, const double *scal, double *parts,
                        hipStream_t st);
kct_status vk_cgls_vol(float *x, void *p, const void *s, int dt, int64_t n, const double *scal, double *parts,
                       hipStream_t st);
kct_status vk_lsqr_vol(float *x, float *w, const void *V, int dt, int64_t n, const double *scal, hipStream_t st);
kct_status vk_lsmr_vol(float *x, float *h, float *hbar, const void *V, int dt, int64_t n, const double *scal,
                       hipStream_t st);
kct_status vk_combine(float *x, const void *basis, int dt, int64_t n, const double *coef, const double *scal,
                      hipStream_t st);

kct_status vk_save_x(const float *x, float *xp, int64_t n, const double *S, hipStream_t st);
kct_status vk_restore_x(float *x, const float *xp, int64_t n, const double *S, hipStream_t st);
kct_status sk_explicit(double *S, Reduced r, double *hist, bool stop, hipStream_t st);
kct_status sk_cgls_init(double *S, Reduced p, double lam, int n_iter, hipStream_t st);
kct_status sk_cgls_alpha(double *S, Reduced q, Reduced p, hipStream_t st);
kct_status sk_cgls_beta(double *S, Reduced s, Reduced r, double *hist, hipStream_t st);
kct_status sk_gk_init1(double *S, Reduced u, double lam, int n_iter, hipStream_t st);
kct_status sk_gk_init2(double *S, Reduced v, double *gk, hipStream_t st);
kct_status sk_gk_beta(double *S, Reduced u, hipStream_t st);
kct_status sk_lsqr_alpha(double *S, Reduced v, double *hist, double *gk, hipStream_t st);
kct_status sk_lsmr_alpha(double *S, Reduced v, double *hist, hipStream_t st);
kct_status sk_hybrid_solve(double *S, const double *gk, double *work, double *coef, hipStream_t st);
kct_status sk_hybrid_choose(double *S, const double *gk, double *work, double *coef, double *hist, int rule,
                            double noise_level, hipStream_t st);
// The same on a dense (k+1) x k matrix M (column-major, leading dimension ldm,
// rows 0..j+1 of column j used), beta_1 = S[S_BETA], coef = y.
kct_status sk_hybrid_choose_dense(double *S, const double *M, int ldm, double *work, double *coef, double *hist,
                                  int rule, double noise_level, hipStream_t st);

// Total variation (IRN-TV).
int tv_num_groups(int64_t M);
kct_status tv_weights(const Plan &p, const float *x, float *Lw, double eps, hipStream_t st);
kct_status tv_grad_norm(const Plan &p, const void *v, int dt, const float *Lw, double lam, const double *S,
                        double *parts, hipStream_t st);
kct_status tv_grad_store(const Plan &p, const void *v, int dt, const float *Lw, float *r2, const double *S, int ci,
                         double c, bool accumulate, hipStream_t st);
kct_status tv_adjoint_add(const Plan &p, void *s, int dt, const float *r2, const float *Lw, double lam,
                          const double *S, double *parts, hipStream_t st);
kct_status sk_tv_restart(double *S, Reduced s, bool first, int n_rows, double lam, hipStream_t st);
kct_status sk_tv_alpha(double *S, Reduced q, Reduced t, double lam, hipStream_t st);

} // namespace kct
