// SIRT and OS-SART, the algebraic reconstruction methods the paper compares
// the Krylov solvers with (Sec. 3): vector and scalar kernels.
//
//   x <- x + lam V_s A_s^T W (b_s - A_s x)     for each ordered subset s
//
// W = 1 / (A 1) (inverse ray lengths), V_s = 1 / (A_s^T 1) (inverse column
// sums of the subset's rows), 0 where a sum vanishes.  SIRT is the case of one
// subset.  The projectors come from the matched pair; these kernels add the
// elementwise weights, the x update and the residual history.

#include "sart.hpp"

#include <algorithm>

namespace kct {

namespace {

__device__ inline double blk_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
    return s;
}

// v = 1 / v where v != 0, else 0.
__global__ __launch_bounds__(256) void k_inv_nz(float *__restrict__ v, int64_t n)
{
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const float a = v[e];
        v[e] = a != 0.f ? 1.f / a : 0.f;
    }
}

// r *= w.
__global__ __launch_bounds__(256) void k_mul(float *__restrict__ r, const float *__restrict__ w, int64_t n)
{
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) r[e] *= w[e];
}

// x += lam V s (nothing once the run is done).
__global__ __launch_bounds__(256) void k_sart_x(float *__restrict__ x, const float *__restrict__ s,
                                                const float *__restrict__ V, int64_t n, const double *__restrict__ S)
{
    if (S[S_DONE] != 0.0) return;
    const float lam = float(S[S_LAMBDA]);
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
        x[e] = fmaf(lam * V[e], s[e], x[e]);
}

__global__ void k_sc_sart_init(double *S, int n_iter, double lam)
{
    if (threadIdx.x != 0) return;
    S[S_ITER] = n_iter;
    S[S_HROW] = 0.0;
    S[S_DONE] = 0.0;
    S[S_RES] = 0.0;
    S[S_LAMBDA] = lam;
    S[S_HLAM] = lam;
}

// Residual history: S_RES accumulates ||b_s - A_s x||^2 over the subsets of
// one sweep; the last subset writes the row [sqrt(S_RES), 0, 0, done, lam].
__global__ __launch_bounds__(256) void k_sc_sart_res(double *S, const double *p, int64_t n, double *hist, int first,
                                                     int last)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += p[e];
    s = blk_sum(s, red);
    if (threadIdx.x != 0) return;
    if (first) S[S_RES] = 0.0;
    if (S[S_DONE] == 0.0) {
        if (s == s && s - s == 0.0) S[S_RES] += s;
        else S[S_DONE] = 2.0;
    }
    if (last) {
        if (hist) {
            const int64_t row = int64_t(S[S_HROW]);
            if (row < int64_t(S[S_ITER])) {
                double *h = hist + row * KCT_HIST_COLS;
                h[0] = sqrt(S[S_RES]);
                h[1] = 0.0;
                h[2] = 0.0;
                h[3] = hist_code(S);
                h[4] = S[S_HLAM];
            }
        }
        S[S_HROW] += 1.0;
    }
}

// Position i of the permuted angle order holds angle k + m j: block k (the
// angles a = k mod m) starts at k q + min(k, r), q = na / m, r = na mod m, and
// holds q + 1 angles when k < r, else q.
__device__ inline int perm_angle(int i, int na, int m)
{
    const int q = na / m, r = na % m;
    int k, j;
    if (i < r * (q + 1)) {
        k = i / (q + 1);
        j = i - k * (q + 1);
    } else {
        const int i2 = i - r * (q + 1);
        k = r + i2 / q;
        j = i2 - (k - r) * q;
    }
    return k + m * j;
}

__global__ __launch_bounds__(256) void k_perm_tab(AngleGeo *__restrict__ out, const AngleGeo *__restrict__ in, int na,
                                                  int m)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < na; i += gridDim.x * 256) out[i] = in[perm_angle(i, na, m)];
}

__global__ __launch_bounds__(256) void k_perm_proj(float *__restrict__ out, const float *__restrict__ in, int na,
                                                   int64_t slab, int m)
{
    const int64_t n = int64_t(na) * slab;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const int i = int(e / slab);
        out[e] = in[int64_t(perm_angle(i, na, m)) * slab + (e - int64_t(i) * slab)];
    }
}

int sa_groups(int64_t n)
{
    const int64_t g = (n + 1023) / 1024;
    return int(std::max<int64_t>(1, std::min<int64_t>(g, 2048)));
}

} // namespace

#define KCT_SA_CHECK(expr)                                                                                         \
    do {                                                                                                           \
        kct_status s_ = (expr);                                                                                    \
        if (s_ != KCT_OK) return s_;                                                                               \
    } while (0)

kct_status sa_inv_nz(float *v, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_inv_nz, dim3(sa_groups(n)), dim3(256), 0, st, v, n);
    return check_hip(hipGetLastError(), "sart inverse");
}

kct_status sa_mul(float *r, const float *w, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_mul, dim3(sa_groups(n)), dim3(256), 0, st, r, w, n);
    return check_hip(hipGetLastError(), "sart weight");
}

kct_status sa_update_x(float *x, const float *s, const float *V, int64_t n, const double *S, hipStream_t st)
{
    hipLaunchKernelGGL(k_sart_x, dim3(sa_groups(n)), dim3(256), 0, st, x, s, V, n, S);
    return check_hip(hipGetLastError(), "sart update");
}

kct_status sa_permute(AngleGeo *tab_out, const AngleGeo *tab_in, float *b_out, const float *b_in, int na, int64_t slab,
                      int m, hipStream_t st)
{
    hipLaunchKernelGGL(k_perm_tab, dim3((na + 255) / 256), dim3(256), 0, st, tab_out, tab_in, na, m);
    KCT_SA_CHECK(check_hip(hipGetLastError(), "permuted table"));
    hipLaunchKernelGGL(k_perm_proj, dim3(sa_groups(int64_t(na) * slab)), dim3(256), 0, st, b_out, b_in, na, slab, m);
    return check_hip(hipGetLastError(), "permuted projections");
}

int sa_block_start(int k, int na, int m)
{
    const int q = na / m, r = na % m;
    return k * q + std::min(k, r);
}

kct_status sa_sc_init(double *S, int n_iter, double lam, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_sart_init, dim3(1), dim3(64), 0, st, S, n_iter, lam);
    return check_hip(hipGetLastError(), "sart init");
}

kct_status sa_sc_res(double *S, const double *p, int64_t n, double *hist, bool first, bool last, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_sart_res, dim3(1), dim3(256), 0, st, S, p, n, hist, first ? 1 : 0, last ? 1 : 0);
    return check_hip(hipGetLastError(), "sart residual");
}

} // namespace kct
