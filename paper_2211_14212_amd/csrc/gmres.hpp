// Internal declarations of the AB-/BA-GMRES kernels and the interpolating
// back projector.
#pragma once

#include "kct_internal.hpp"

namespace kct {

constexpr int GM_GROUPS = 2048; // workgroups of the GMRES vector kernels

int gm_num_groups(int64_t n);
kct_status gm_dot(const void *a, const void *b, int dt, int64_t n, double *parts, hipStream_t st);
kct_status gm_axpy(void *w, const void *v, int dt, int64_t n, const double *S, int ci, hipStream_t st);
kct_status gm_scale(void *w, int dt, int64_t n, const double *S, int ci, hipStream_t st);
kct_status gm_sc_init(double *S, const double *p, int64_t n, double *g, int n_iter, hipStream_t st);
kct_status gm_sc_h(double *S, const double *p, int64_t n, double *H, int i, int j, int ldh, hipStream_t st);
kct_status gm_sc_norm(double *S, const double *p, int64_t n, double *H, int j, int ldh, hipStream_t st);
kct_status gm_sc_givens(double *S, double *H, double *cs, double *sn, double *g, int j, int ldh, double *hist,
                        hipStream_t st);
kct_status gm_sc_solve(const double *S, const double *H, const double *g, double *coef, int ldh, hipStream_t st);

int64_t ibp_num_groups(const Plan &p);
kct_status launch_interp_backward(Plan &p, const void *proj, int proj_dtype, void *vol, int vol_dtype,
                                  const Epilogue &ep, hipStream_t st);

} // namespace kct
