// Internal declarations of the SIRT / OS-SART kernels.
#pragma once

#include "kct_internal.hpp"

namespace kct {

kct_status sa_inv_nz(float *v, int64_t n, hipStream_t st);
kct_status sa_mul(float *r, const float *w, int64_t n, hipStream_t st);
kct_status sa_update_x(float *x, const float *s, const float *V, int64_t n, const double *S, hipStream_t st);
kct_status sa_sc_init(double *S, int n_iter, double lam, hipStream_t st);
// The angles in the order k, k + m, k + 2m, ... for k = 0..m-1 (table and
// projection slabs of `slab` values), and the first position of block k.
kct_status sa_permute(AngleGeo *tab_out, const AngleGeo *tab_in, float *b_out, const float *b_in, int na, int64_t slab,
                      int m, hipStream_t st);
int sa_block_start(int k, int na, int m);
kct_status sa_sc_res(double *S, const double *p, int64_t n, double *hist, bool first, bool last, hipStream_t st);

} // namespace kct
