// AB- and BA-GMRES building blocks (paper Sec. 2.1.4), gfx950.
//
// GMRES on the operator AB (AB-GMRES, B a right preconditioner, basis in
// projection space) or BA (BA-GMRES, B a left preconditioner, basis in volume
// space), for a back projector B that need not be A^T.  Arnoldi with modified
// Gram-Schmidt keeps the basis V_1..V_{k+1} (unit vectors, stored in the
// solver's vector type) and the (k+1) x k Hessenberg matrix H in device FP64.
// Givens rotations reduce H to triangular form as columns arrive, so the
// residual norm |g_{k+1}| of the small problem min ||beta e_1 - H y|| is known
// every iteration; y is found by back substitution at the end.
//
// Vector kernels read FP32, BF16 or FP16 and accumulate dot products in FP64
// per workgroup (fixed order); scalar kernels run on one thread.

#include "gmres.hpp"

#include <algorithm>

namespace kct {

namespace {

__device__ inline double wave_block_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
    return s;
}

__device__ inline double sum_parts(const double *p, int64_t n, double *red)
{
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += p[e];
    return wave_block_sum(s, red);
}

__device__ inline bool finite(double v) { return v == v && v - v == 0.0; }

// parts[workgroup] = sum over its elements of a_e * b_e (FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                             double *__restrict__ parts)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
        s += double(to_f32(a[e])) * double(to_f32(b[e]));
    s = wave_block_sum(s, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

// w += S[ci] * v.
template <typename T>
__global__ __launch_bounds__(256) void k_axpy_s(T *__restrict__ w, const T *__restrict__ v, int64_t n,
                                                const double *__restrict__ S, int ci)
{
    const float c = float(S[ci]);
    if (c == 0.f) return;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
        w[e] = from_f32<T>(fmaf(c, to_f32(v[e]), to_f32(w[e])));
}

// w *= S[ci].
template <typename T>
__global__ __launch_bounds__(256) void k_scale_s(T *__restrict__ w, int64_t n, const double *__restrict__ S, int ci)
{
    const float c = float(S[ci]);
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
        w[e] = from_f32<T>(c * to_f32(w[e]));
}

// Start: beta = ||r0||, V_1 = r0 / beta (scale factor left in S_V0), g_1 = beta.
__global__ __launch_bounds__(256) void k_sc_gm_init(double *S, const double *p, int64_t n, double *g, int n_iter)
{
    __shared__ double red[4];
    const double b2 = sum_parts(p, n, red);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(b2);
    S[S_ITER] = n_iter;
    S[S_HROW] = 0.0;
    S[S_KGK] = 0.0;
    S[S_HLAM] = 0.0;
    S[S_BETA] = beta;
    S[S_DONE] = !finite(beta) ? 2.0 : (beta > 0.0 ? 0.0 : 1.0);
    S[S_V0] = S[S_DONE] == 0.0 ? 1.0 / beta : 0.0;
    g[0] = S[S_DONE] == 0.0 ? beta : 0.0;
}

// Modified Gram-Schmidt step: H[i, j] = <w, V_i>; S_P0 = -H[i, j] for w -= H[i, j] V_i.
__global__ __launch_bounds__(256) void k_sc_gm_h(double *S, const double *p, int64_t n, double *H, int i, int j,
                                                 int ldh)
{
    __shared__ double red[4];
    const double h = sum_parts(p, n, red);
    if (threadIdx.x != 0) return;
    const bool live = S[S_DONE] == 0.0 && finite(h);
    if (S[S_DONE] == 0.0 && !finite(h)) S[S_DONE] = 2.0;
    H[int64_t(j) * ldh + i] = live ? h : 0.0;
    S[S_P0] = live ? -h : 0.0;
}

// H[j+1, j] = ||w||; S_V0 = 1 / ||w|| normalises it into V_{j+1}.  A zero
// norm means the Krylov space is invariant: the small problem is then solved
// exactly and the run stops here (done = 1).
__global__ __launch_bounds__(256) void k_sc_gm_norm(double *S, const double *p, int64_t n, double *H, int j,
                                                    int ldh)
{
    __shared__ double red[4];
    const double h2 = sum_parts(p, n, red);
    if (threadIdx.x != 0) return;
    const double h = sqrt(h2);
    S[S_V0] = 0.0;
    if (S[S_DONE] != 0.0) return;
    if (!finite(h)) {
        S[S_DONE] = 2.0;
        return;
    }
    H[int64_t(j) * ldh + j + 1] = h;
    S[S_KGK] = j + 1; // columns of H in use
    if (h > 0.0) S[S_V0] = 1.0 / h;
}

// Givens rotations: apply the previous ones to column j of H, make the new one
// zero H[j+1, j], rotate g; history row j: [|g_{j+2}|, H[j+1, j] (before
// rotation), R[j, j], done, 0].
__global__ void k_sc_gm_givens(double *S, double *H, double *cs, double *sn, double *g, int j, int ldh,
                               double *hist)
{
    if (threadIdx.x != 0) return;
    double sub = 0.0, diag = 0.0;
    if (S[S_DONE] != 2.0 && int(S[S_KGK]) == j + 1) {
        double *h = H + int64_t(j) * ldh;
        for (int i = 0; i < j; ++i) {
            const double a = h[i], b = h[i + 1];
            h[i] = cs[i] * a + sn[i] * b;
            h[i + 1] = -sn[i] * a + cs[i] * b;
        }
        sub = h[j + 1];
        const double r = hypot(h[j], h[j + 1]);
        const double c = r > 0.0 ? h[j] / r : 1.0, s = r > 0.0 ? h[j + 1] / r : 0.0;
        cs[j] = c;
        sn[j] = s;
        h[j] = r;
        h[j + 1] = 0.0;
        const double gj = g[j];
        g[j] = c * gj;
        g[j + 1] = -s * gj;
        diag = r;
        if (sub == 0.0) S[S_DONE] = 1.0;
    }
    const int kk = int(S[S_KGK]);
    if (hist) {
        const int64_t row = int64_t(S[S_HROW]);
        if (row < int64_t(S[S_ITER])) {
            double *o = hist + row * KCT_HIST_COLS;
            o[0] = kk > 0 ? fabs(g[kk]) : S[S_BETA];
            o[1] = sub;
            o[2] = diag;
            o[3] = hist_code(S);
            o[4] = 0.0;
        }
    }
    S[S_HROW] += 1.0;
}

// y = R^-1 g (back substitution over the k columns in use).
__global__ void k_sc_gm_solve(const double *S, const double *H, const double *g, double *coef, int ldh)
{
    if (threadIdx.x != 0) return;
    const int kk = int(S[S_KGK]);
    for (int c = 0; c < kk; ++c) coef[c] = 0.0; // x = 0 after a non-finite scalar
    const int k = S[S_DONE] == 2.0 ? 0 : kk;
    for (int c = k - 1; c >= 0; --c) {
        double v = g[c];
        for (int cc = c + 1; cc < k; ++cc) v -= H[int64_t(cc) * ldh + c] * coef[cc];
        const double d = H[int64_t(c) * ldh + c];
        coef[c] = d != 0.0 ? v / d : 0.0;
    }
}

int gm_groups(int64_t n)
{
    const int64_t g = (n + 1023) / 1024;
    return int(std::max<int64_t>(1, std::min<int64_t>(g, GM_GROUPS)));
}

} // namespace

#define KCT_GM_DISPATCH(dt, T, ...)                                                                                \
    switch (dt) {                                                                                                  \
    case KCT_F32: { using T = float; __VA_ARGS__; } break;                                                        \
    case KCT_BF16: { using T = bf16; __VA_ARGS__; } break;                                                        \
    case KCT_F16: { using T = _Float16; __VA_ARGS__; } break;                                                     \
    default: return fail(KCT_E_DTYPE, "unsupported storage type");                                               \
    }

int gm_num_groups(int64_t n) { return gm_groups(n); }

kct_status gm_dot(const void *a, const void *b, int dt, int64_t n, double *parts, hipStream_t st)
{
    KCT_GM_DISPATCH(dt, T, hipLaunchKernelGGL(k_dot<T>, dim3(gm_groups(n)), dim3(256), 0, st,
                                              static_cast<const T *>(a), static_cast<const T *>(b), n, parts));
    return check_hip(hipGetLastError(), "gmres dot");
}

kct_status gm_axpy(void *w, const void *v, int dt, int64_t n, const double *S, int ci, hipStream_t st)
{
    KCT_GM_DISPATCH(dt, T, hipLaunchKernelGGL(k_axpy_s<T>, dim3(gm_groups(n)), dim3(256), 0, st, static_cast<T *>(w),
                                              static_cast<const T *>(v), n, S, ci));
    return check_hip(hipGetLastError(), "gmres axpy");
}

kct_status gm_scale(void *w, int dt, int64_t n, const double *S, int ci, hipStream_t st)
{
    KCT_GM_DISPATCH(dt, T, hipLaunchKernelGGL(k_scale_s<T>, dim3(gm_groups(n)), dim3(256), 0, st,
                                              static_cast<T *>(w), n, S, ci));
    return check_hip(hipGetLastError(), "gmres scale");
}

kct_status gm_sc_init(double *S, const double *p, int64_t n, double *g, int n_iter, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_gm_init, dim3(1), dim3(256), 0, st, S, p, n, g, n_iter);
    return check_hip(hipGetLastError(), "gmres init");
}

kct_status gm_sc_h(double *S, const double *p, int64_t n, double *H, int i, int j, int ldh, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_gm_h, dim3(1), dim3(256), 0, st, S, p, n, H, i, j, ldh);
    return check_hip(hipGetLastError(), "gmres h");
}

kct_status gm_sc_norm(double *S, const double *p, int64_t n, double *H, int j, int ldh, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_gm_norm, dim3(1), dim3(256), 0, st, S, p, n, H, j, ldh);
    return check_hip(hipGetLastError(), "gmres norm");
}

kct_status gm_sc_givens(double *S, double *H, double *cs, double *sn, double *g, int j, int ldh, double *hist,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_gm_givens, dim3(1), dim3(64), 0, st, S, H, cs, sn, g, j, ldh, hist);
    return check_hip(hipGetLastError(), "gmres givens");
}

kct_status gm_sc_solve(const double *S, const double *H, const double *g, double *coef, int ldh, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_gm_solve, dim3(1), dim3(64), 0, st, S, H, g, coef, ldh);
    return check_hip(hipGetLastError(), "gmres solve");
}

} // namespace kct
