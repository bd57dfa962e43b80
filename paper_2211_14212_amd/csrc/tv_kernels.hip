// Total-variation operators of IRN-TV (paper Sec. 2.3, eqs. (TV),
// (TV_reweighted), (TV_approx)), gfx950.
//
// D is the forward difference along x, y and z with unit spacing and a zero
// difference at the last index of each axis (Neumann boundary; the paper
// leaves the boundary condition open).  D^T is its exact adjoint.  The IRN
// weights are L = diag(w^{-1/2}) with w = sqrt(|D x|^2 + eps^2) per voxel,
// applied to all three gradient components of that voxel.  The gradient-space
// residual r2 is stored planar: component c of voxel e at r2[c*M + e].
//
// All kernels are one thread per voxel, one workgroup per x-row at a time
// (neighbour reads along x are contiguous, along y and z one row or slice
// away, all coalesced across a wave), and bound by HBM bandwidth.

#include "krylov.hpp"

namespace kct {

namespace {

__device__ inline double block_sum_tv(double v)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

struct Dims {
    int nx, ny, nz;
    int64_t M;
};

// The kernels walk x-rows: workgroups stride over the ny*nz rows and the
// threads over x, so voxel (i, j, k) costs one division per row instead of a
// 64-bit division and modulo per voxel.  The row order is XCD-aware:
// workgroup b runs on XCD b mod 8 (the grid is a multiple of 8) and each XCD
// walks one contiguous eighth of the rows, so the z neighbours of a row (one
// slice away) are mostly read through the same L2.
#define TV_ROWS(d)                                                                                                 \
    for (int64_t rows = int64_t(d.ny) * d.nz, per = (rows + 7) / 8, xcd = blockIdx.x & 7,                        \
                 end = rows < (xcd + 1) * per ? rows : (xcd + 1) * per, row = xcd * per + (blockIdx.x >> 3);      \
         row < end; row += gridDim.x >> 3)

template <typename T>
__device__ inline void grad_at(const T *x, Dims d, int64_t e, int i, int j, int k, float &gx, float &gy, float &gz)
{
    // The neighbour past the last index is the voxel itself (difference
    // exactly 0), so the loads are unconditional and issue together.
    const int64_t sxy = int64_t(d.nx) * d.ny;
    const float c = to_f32(x[e]);
    const float xp = to_f32(x[e + (i < d.nx - 1 ? 1 : 0)]);
    const float yp = to_f32(x[e + (j < d.ny - 1 ? d.nx : 0)]);
    const float zp = to_f32(x[e + (k < d.nz - 1 ? sxy : 0)]);
    gx = xp - c;
    gy = yp - c;
    gz = zp - c;
}

// Lw = (|D x|^2 + eps^2)^{-1/4}.
__global__ __launch_bounds__(256) void k_tv_weights(const float *__restrict__ x, float *__restrict__ Lw, Dims d,
                                                    double eps)
{
    TV_ROWS(d)
    {
        const int j = int(row % d.ny), k = int(row / d.ny);
        for (int i = threadIdx.x; i < d.nx; i += 256) {
            const int64_t e = row * d.nx + i;
            float gx, gy, gz;
            grad_at(x, d, e, i, j, k, gx, gy, gz);
            const double w = sqrt(double(gx) * gx + double(gy) * gy + double(gz) * gz + eps * eps);
            Lw[e] = float(1.0 / sqrt(w));
        }
    }
}

// Partial sums of |lam L D p|^2.
template <typename T>
__global__ __launch_bounds__(256) void k_tv_grad_norm(const T *__restrict__ p, const float *__restrict__ Lw, Dims d,
                                                      double lam, const double *S, double *parts)
{
    double s = 0.0;
    if (S[S_DONE] == 0.0) {
        TV_ROWS(d)
        {
            const int j = int(row % d.ny), k = int(row / d.ny);
            for (int i = threadIdx.x; i < d.nx; i += 256) {
                const int64_t e = row * d.nx + i;
                float gx, gy, gz;
                grad_at(p, d, e, i, j, k, gx, gy, gz);
                const double l = lam * double(Lw[e]);
                s += l * l * (double(gx) * gx + double(gy) * gy + double(gz) * gz);
            }
        }
    }
    s = block_sum_tv(s);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

// r2 = c * L D v (assign) or r2 += c * L D v (accumulate); c = S[ci] or cgiven.
template <typename T>
__global__ __launch_bounds__(256) void k_tv_grad_store(const T *__restrict__ v, const float *__restrict__ Lw, Dims d,
                                                       float *__restrict__ r2, const double *S, int ci, double cgiven,
                                                       int accumulate)
{
    const double c = ci >= 0 ? S[ci] : cgiven;
    if (accumulate && c == 0.0) return;
    TV_ROWS(d)
    {
        const int j = int(row % d.ny), k = int(row / d.ny);
        for (int i = threadIdx.x; i < d.nx; i += 256) {
            const int64_t e = row * d.nx + i;
            float gx, gy, gz;
            grad_at(v, d, e, i, j, k, gx, gy, gz);
            const double l = c * double(Lw[e]);
            if (accumulate) {
                r2[e] = float(double(r2[e]) + l * gx);
                r2[d.M + e] = float(double(r2[d.M + e]) + l * gy);
                r2[2 * d.M + e] = float(double(r2[2 * d.M + e]) + l * gz);
            } else {
                r2[e] = float(l * gx);
                r2[d.M + e] = float(l * gy);
                r2[2 * d.M + e] = float(l * gz);
            }
        }
    }
}

// s += lam D^T (L r2); partial sums of s^2.
template <typename T>
__global__ __launch_bounds__(256) void k_tv_adjoint_add(T *__restrict__ s, const float *__restrict__ r2,
                                                        const float *__restrict__ Lw, Dims d, double lam,
                                                        const double *S, double *parts)
{
    double acc = 0.0;
    const bool skip = S && S[S_DONE] != 0.0;
    const int64_t sxy = int64_t(d.nx) * d.ny;
    if (!skip) {
        TV_ROWS(d)
        {
            const int j = int(row % d.ny), k = int(row / d.ny);
            // Terms of missing neighbours are multiplied by 0 rather than
            // skipped, so the loads are unconditional (clamped to the voxel).
            const double fyp = j < d.ny - 1 ? 1.0 : 0.0, fym = j > 0 ? 1.0 : 0.0;
            const double fzp = k < d.nz - 1 ? 1.0 : 0.0, fzm = k > 0 ? 1.0 : 0.0;
            const int64_t dym = j > 0 ? d.nx : 0, dzm = k > 0 ? sxy : 0;
            for (int i = threadIdx.x; i < d.nx; i += 256) {
                const int64_t e = row * d.nx + i;
                const double fxp = i < d.nx - 1 ? 1.0 : 0.0, fxm = i > 0 ? 1.0 : 0.0;
                const int64_t dxm = i > 0 ? 1 : 0;
                const double le = Lw[e];
                const double gx = r2[e], gy = r2[d.M + e], gz = r2[2 * d.M + e];
                const double gxm = r2[e - dxm], gym = r2[d.M + e - dym], gzm = r2[2 * d.M + e - dzm];
                const double lx = Lw[e - dxm], ly = Lw[e - dym], lz = Lw[e - dzm];
                double t = 0.0;
                t -= fxp * (le * gx);
                t += fxm * (lx * gxm);
                t -= fyp * (le * gy);
                t += fym * (ly * gym);
                t -= fzp * (le * gz);
                t += fzm * (lz * gzm);
                const T o = from_f32<T>(float(double(to_f32(s[e])) + lam * t));
                s[e] = o;
                const double f = to_f32(o);
                acc += f * f;
            }
        }
    }
    acc = block_sum_tv(acc);
    if (threadIdx.x == 0 && parts) parts[blockIdx.x] = acc;
}

// IRN restart of CGLS: gamma = ||s||^2, fresh Krylov space.
__global__ __launch_bounds__(256) void k_sc_tv_restart(double *S, const double *ps, int64_t ns, int first,
                                                       int n_rows, double lam)
{
    double s2 = 0.0;
    for (int64_t e = threadIdx.x; e < ns; e += 256) s2 += ps[e];
    s2 = block_sum_tv(s2);
    if (threadIdx.x != 0) return;
    if (first) {
        S[S_HROW] = 0.0;
        S[S_ITER] = n_rows;
        S[S_RES] = 0.0;
        S[S_DONE] = 0.0;
        S[S_HLAM] = lam;
    }
    if (S[S_DONE] != 2.0) S[S_DONE] = (s2 == s2 && s2 - s2 == 0.0) ? (s2 > 0.0 ? 0.0 : 1.0) : 2.0;
    S[S_GAMMA] = s2;
    S[S_LAMBDA] = 0.0;
}

// IRN inner CGLS: delta = ||A p||^2 + ||lam L D p||^2, alpha = gamma / delta.
__global__ __launch_bounds__(256) void k_sc_tv_alpha(double *S, const double *pq, int64_t nq, const double *pt,
                                                     int64_t nt, double lam)
{
    double q2 = 0.0, t2 = 0.0;
    for (int64_t e = threadIdx.x; e < nq; e += 256) q2 += pq[e];
    q2 = block_sum_tv(q2);
    for (int64_t e = threadIdx.x; e < nt; e += 256) t2 += pt[e];
    t2 = block_sum_tv(t2);
    if (threadIdx.x != 0) return;
    double alpha = 0.0;
    if (S[S_DONE] == 0.0) {
        const double delta = q2 + t2;
        if (delta > 0.0 && delta - delta == 0.0) alpha = S[S_GAMMA] / delta;
        else S[S_DONE] = (delta - delta == 0.0) ? 1.0 : 2.0;
    }
    S[S_ALPHA] = alpha;
    S[S_P0] = -alpha;        // r1 += P0 q1
    S[S_V3] = -alpha * lam;  // r2 += V3 L D p
}

// A multiple of 8 workgroups (the XCD-aware row order needs it).
int tv_groups(int64_t n)
{
    const int64_t g = (n + 1023) / 1024;
    return int(std::max<int64_t>(8, std::min<int64_t>((g + 7) / 8 * 8, VEC_GROUPS)));
}

} // namespace

#define KCT_TV_DISPATCH(dt, T, ...)                                                                                \
    switch (dt) {                                                                                                  \
    case KCT_F32: { using T = float; __VA_ARGS__; } break;                                                        \
    case KCT_BF16: { using T = bf16; __VA_ARGS__; } break;                                                        \
    case KCT_F16: { using T = _Float16; __VA_ARGS__; } break;                                                     \
    default: return fail(KCT_E_DTYPE, "unsupported storage type");                                               \
    }

static Dims dims(const Plan &p) { return Dims{p.gp.nx, p.gp.ny, p.gp.nz, p.n_vox()}; }

kct_status tv_weights(const Plan &p, const float *x, float *Lw, double eps, hipStream_t st)
{
    const Dims d = dims(p);
    hipLaunchKernelGGL(k_tv_weights, dim3(tv_groups(d.M)), dim3(256), 0, st, x, Lw, d, eps);
    return check_hip(hipGetLastError(), "tv weights");
}

kct_status tv_grad_norm(const Plan &p, const void *v, int dt, const float *Lw, double lam, const double *S,
                        double *parts, hipStream_t st)
{
    const Dims d = dims(p);
    KCT_TV_DISPATCH(dt, T, hipLaunchKernelGGL(k_tv_grad_norm<T>, dim3(tv_groups(d.M)), dim3(256), 0, st,
                                              static_cast<const T *>(v), Lw, d, lam, S, parts));
    return check_hip(hipGetLastError(), "tv gradient norm");
}

kct_status tv_grad_store(const Plan &p, const void *v, int dt, const float *Lw, float *r2, const double *S, int ci,
                         double c, bool accumulate, hipStream_t st)
{
    const Dims d = dims(p);
    KCT_TV_DISPATCH(dt, T, hipLaunchKernelGGL(k_tv_grad_store<T>, dim3(tv_groups(d.M)), dim3(256), 0, st,
                                              static_cast<const T *>(v), Lw, d, r2, S, ci, c, accumulate ? 1 : 0));
    return check_hip(hipGetLastError(), "tv gradient");
}

kct_status tv_adjoint_add(const Plan &p, void *s, int dt, const float *r2, const float *Lw, double lam,
                          const double *S, double *parts, hipStream_t st)
{
    const Dims d = dims(p);
    KCT_TV_DISPATCH(dt, T, hipLaunchKernelGGL(k_tv_adjoint_add<T>, dim3(tv_groups(d.M)), dim3(256), 0, st,
                                              static_cast<T *>(s), r2, Lw, d, lam, S, parts));
    return check_hip(hipGetLastError(), "tv adjoint");
}

int tv_num_groups(int64_t M) { return tv_groups(M); }

kct_status sk_tv_restart(double *S, Reduced s, bool first, int n_rows, double lam, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_tv_restart, dim3(1), dim3(256), 0, st, S, s.ptr, s.n, first ? 1 : 0, n_rows, lam);
    return check_hip(hipGetLastError(), "tv restart scalars");
}

kct_status sk_tv_alpha(double *S, Reduced q, Reduced t, double lam, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_tv_alpha, dim3(1), dim3(256), 0, st, S, q.ptr, q.n, t.ptr, t.n, lam);
    return check_hip(hipGetLastError(), "tv alpha");
}

} // namespace kct
