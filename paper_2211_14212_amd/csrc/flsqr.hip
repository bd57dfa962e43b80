// Hybrid fLSQR-TV (paper Sec. 2.3.2, eq. (TV_standard_form)): vector and
// scalar kernels of the standard-form transform and of the inner CG.
//
// The TV weights L (one factor per voxel, shared by the three gradient
// components) define the changing preconditioner P = E (L D)^+ with
//   (L D)^+ v = K^+ D^T L v,   K = D^T L^2 D (weighted Neumann Laplacian),
//   E z = z - 1 (g^T z) / (a^T a),   a = A 1, g = A^T a,
// and its transpose P^T w = L D K^+ E^T w with E^T w = w - g (1^T w)/(a^T a).
// K^+ is applied by CG from zero on the complement of the constants, where K
// is SPD: every step removes the mean of the residual (folded into the
// direction update), so rounding cannot drive the iterate along the null
// space.  The CG's vectors and stencil arithmetic are FP64: with weights near
// 1/sqrt(eps) in flat regions K is badly conditioned, and an FP32 CG moved
// the 4th fLSQR-TV iterate of the 32^3 workload at eps = 1e-3 by 1.1e-3 in
// oracle runs, five times the effect of FP32 rounding of the matvecs.  Its
// right-hand side arrives in FP32 and its result leaves in FP32.  D is the forward difference with a zero last difference per axis,
// as in IRN-TV.  Volumes are x-fastest; gradient-space vectors are planar
// (component c of voxel e at c*M + e).  The vector kernels are one thread per
// voxel in a grid-stride loop, the stencils one workgroup per x-row; all are
// bound by HBM bandwidth, with the six neighbours' reads served by L2.

#include "flsqr.hpp"

#include <algorithm>

namespace kct {

namespace {

struct Dims {
    int nx, ny, nz;
    int64_t M;
};

Dims dims(const Plan &p) { return Dims{p.gp.nx, p.gp.ny, p.gp.nz, p.n_vox()}; }

// Fixed-order block sum (4 waves of 64).
__device__ inline double block_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// Fixed-order sum of n partials by one workgroup (result on thread 0).
__device__ inline double sum_parts(const double *p, int64_t n, double *red)
{
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += p[e];
    return block_sum(s, red);
}

__device__ inline bool finite(double v) { return v == v && v - v == 0.0; }

#define FL_LOOP(e, n) for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < (n); e += int64_t(gridDim.x) * 256)

// The stencil kernels walk x-rows: workgroups stride over the ny*nz rows and
// the threads over x, so the voxel coordinates cost one division per row
// instead of a 64-bit division and modulo per voxel.  The row order is
// XCD-aware: workgroup b runs on XCD b mod 8 (the grid is a multiple of 8) and
// each XCD walks one contiguous eighth of the rows, so the z neighbours of a
// row (one slice away) are mostly read through the same L2.

__global__ __launch_bounds__(256) void k_fl_lap(const double *__restrict__ p, const float *__restrict__ Lw, Dims d,
                                                double *__restrict__ q, double *parts)
{
    __shared__ double red[4];
    const int64_t sxy = int64_t(d.nx) * d.ny;
    const int64_t rows = int64_t(d.ny) * d.nz;
    double acc = 0.0;
    const int64_t per = (rows + 7) / 8, xcd = blockIdx.x & 7;
    const int64_t end = rows < (xcd + 1) * per ? rows : (xcd + 1) * per;
    for (int64_t row = xcd * per + (blockIdx.x >> 3); row < end; row += gridDim.x >> 3) {
        const int j = int(row % d.ny), k = int(row / d.ny);
        const int64_t e0 = row * d.nx;
        // A missing neighbour (at the boundary) is the voxel itself, so its
        // difference is exactly 0: every load is unconditional and they all
        // issue before the first use.
        const int64_t dyp = j < d.ny - 1 ? d.nx : 0, dym = j > 0 ? d.nx : 0;
        const int64_t dzp = k < d.nz - 1 ? sxy : 0, dzm = k > 0 ? sxy : 0;
        for (int i = threadIdx.x; i < d.nx; i += 256) {
            const int64_t e = e0 + i;
            const int64_t dxp = i < d.nx - 1 ? 1 : 0, dxm = i > 0 ? 1 : 0;
            const double c = p[e], le = Lw[e], we = le * le;
            const double pxp = p[e + dxp], pxm = p[e - dxm], pyp = p[e + dyp], pym = p[e - dym];
            const double pzp = p[e + dzp], pzm = p[e - dzm];
            const double lx = Lw[e - dxm], ly = Lw[e - dym], lz = Lw[e - dzm];
            double t = 0.0;
            t -= we * (pxp - c);
            t += lx * lx * (c - pxm);
            t -= we * (pyp - c);
            t += ly * ly * (c - pym);
            t -= we * (pzp - c);
            t += lz * lz * (c - pzm);
            q[e] = t;
            acc += c * t;
        }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_fl_cg_update(double *__restrict__ t, double *__restrict__ r,
                                                      const double *__restrict__ p, const double *__restrict__ q,
                                                      int64_t n, const double *S, double *psum, double *psq)
{
    __shared__ double red[4];
    const double alpha = S[S_CG_ALPHA];
    double s1 = 0.0, s2 = 0.0;
    FL_LOOP(e, n)
    {
        t[e] = t[e] + alpha * p[e];
        const double v = r[e] - alpha * q[e];
        r[e] = v;
        s1 += v;
        s2 += v * v;
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        psum[blockIdx.x] = s1;
        psq[blockIdx.x] = s2;
    }
}

// First call (rhs given): r = rhs - mu, p = r, t = 0.  Later: r -= mu,
// p = r + beta p.
__global__ __launch_bounds__(256) void k_fl_cg_dir(double *__restrict__ r, double *__restrict__ p,
                                                   double *__restrict__ t, const float *__restrict__ rhs,
                                                   int64_t n, const double *S)
{
    const double mu = S[S_CG_MU], beta = S[S_CG_BETA];
    FL_LOOP(e, n)
    {
        if (rhs) {
            const double v = double(rhs[e]) - mu;
            r[e] = v;
            p[e] = v;
            t[e] = 0.0;
        } else {
            const double v = r[e] - mu;
            r[e] = v;
            p[e] = v + beta * p[e];
        }
    }
}

__global__ __launch_bounds__(256) void k_fl_to_f32(float *__restrict__ out, const double *__restrict__ in, int64_t n)
{
    FL_LOOP(e, n) out[e] = float(in[e]);
}

__global__ __launch_bounds__(256) void k_fl_dtl(const float *__restrict__ v3, const float *__restrict__ Lw, Dims d,
                                                float *__restrict__ out, double *psum, double *psq)
{
    __shared__ double red[4];
    const int64_t sxy = int64_t(d.nx) * d.ny;
    const int64_t rows = int64_t(d.ny) * d.nz;
    double s1 = 0.0, s2 = 0.0;
    const int64_t per = (rows + 7) / 8, xcd = blockIdx.x & 7;
    const int64_t end = rows < (xcd + 1) * per ? rows : (xcd + 1) * per;
    for (int64_t row = xcd * per + (blockIdx.x >> 3); row < end; row += gridDim.x >> 3) {
        const int j = int(row % d.ny), k = int(row / d.ny);
        const int64_t e0 = row * d.nx;
        // Terms of missing neighbours are multiplied by 0 instead of skipped,
        // so every load is unconditional (in bounds: the index is clamped to
        // the voxel itself).
        const float fyp = j < d.ny - 1 ? 1.f : 0.f, fym = j > 0 ? 1.f : 0.f;
        const float fzp = k < d.nz - 1 ? 1.f : 0.f, fzm = k > 0 ? 1.f : 0.f;
        const int64_t dym = j > 0 ? d.nx : 0, dzm = k > 0 ? sxy : 0;
        for (int i = threadIdx.x; i < d.nx; i += 256) {
            const int64_t e = e0 + i;
            const float fxp = i < d.nx - 1 ? 1.f : 0.f, fxm = i > 0 ? 1.f : 0.f;
            const int64_t dxm = i > 0 ? 1 : 0;
            const float le = Lw[e];
            const float gx = v3[e], gy = v3[d.M + e], gz = v3[2 * d.M + e];
            const float gxm = v3[e - dxm], gym = v3[d.M + e - dym], gzm = v3[2 * d.M + e - dzm];
            const float lx = Lw[e - dxm], ly = Lw[e - dym], lz = Lw[e - dzm];
            float t = 0.f;
            t -= fxp * (le * gx);
            t += fxm * (lx * gxm);
            t -= fyp * (le * gy);
            t += fym * (ly * gym);
            t -= fzp * (le * gz);
            t += fzm * (lz * gzm);
            out[e] = t;
            s1 += t;
            s2 += double(t) * t;
        }
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        psum[blockIdx.x] = s1;
        psq[blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(256) void k_fl_sum(const float *__restrict__ v, int64_t n, double *parts)
{
    __shared__ double red[4];
    double s = 0.0;
    FL_LOOP(e, n) s += v[e];
    s = block_sum(s, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fl_axpy_sum(float *__restrict__ r, const float *__restrict__ g, int64_t n,
                                                     const double *S, int ci, double *psum, double *psq)
{
    __shared__ double red[4];
    const double c = S[ci];
    double s1 = 0.0, s2 = 0.0;
    FL_LOOP(e, n)
    {
        const float v = float(double(r[e]) - c * g[e]);
        r[e] = v;
        s1 += v;
        s2 += double(v) * v;
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        psum[blockIdx.x] = s1;
        psq[blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(256) void k_fl_shift(float *__restrict__ out, const float *__restrict__ in, int64_t n,
                                                  const double *S, int ci)
{
    const double c = S[ci];
    FL_LOOP(e, n) out[e] = float(double(in[e]) - c);
}

__global__ __launch_bounds__(256) void k_fl_fill_s(float *__restrict__ out, int64_t n, const double *S, int ci)
{
    const float c = float(S[ci]);
    FL_LOOP(e, n) out[e] = c;
}

__global__ __launch_bounds__(256) void k_fl_bbar(float *__restrict__ out, const float *__restrict__ b,
                                                 const float *__restrict__ a, int64_t n, const double *S,
                                                 double *parts)
{
    __shared__ double red[4];
    const double c = S[S_P0];
    double s = 0.0;
    FL_LOOP(e, n)
    {
        const float v = float(double(b[e]) + c * a[e]);
        out[e] = v;
        s += double(v) * v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fl_combine(float *__restrict__ x, const float *__restrict__ Z, int64_t n,
                                                    const double *__restrict__ coef, const double *S)
{
    const int k = int(S[S_KGK]);
    const double c0 = S[S_FL_C0];
    FL_LOOP(e, n)
    {
        double s = c0;
        for (int i = 0; i < k; ++i) s += coef[i] * double(Z[int64_t(i) * n + e]);
        x[e] = float(s);
    }
}

// ------------------------------------------------------------ scalar kernels

// x0 = c0 1 with c0 = a^T b / a^T a (0 when A 1 = 0); S_P0 = -c0 for bbar.
__global__ __launch_bounds__(256) void k_sc_fl_init(double *S, const double *pca, int64_t nca, const double *pab,
                                                    int64_t nab, int n_iter, double lam)
{
    __shared__ double red[4];
    const double ca = sum_parts(pca, nca, red);
    const double ab = sum_parts(pab, nab, red);
    if (threadIdx.x != 0) return;
    const double c0 = ca > 0.0 ? ab / ca : 0.0;
    S[S_ITER] = n_iter;
    S[S_HROW] = 0.0;
    S[S_KGK] = 0.0;
    S[S_DONE] = finite(c0) ? 0.0 : 2.0;
    S[S_LAMBDA] = lam;
    S[S_HLAM] = lam;
    S[S_FL_CA] = ca;
    S[S_FL_C0] = finite(c0) ? c0 : 0.0;
    S[S_P0] = finite(c0) ? -c0 : 0.0;
}

// beta_1 = ||bbar||; S_V0 = 1 / beta_1 normalises u_1.
__global__ __launch_bounds__(256) void k_sc_fl_beta1(double *S, const double *p, int64_t n)
{
    __shared__ double red[4];
    const double b2 = sum_parts(p, n, red);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(b2);
    S[S_BETA] = beta;
    if (S[S_DONE] == 0.0) S[S_DONE] = !finite(beta) ? 2.0 : (beta > 0.0 ? 0.0 : 1.0);
    S[S_V0] = S[S_DONE] == 0.0 ? 1.0 / beta : 0.0;
}

// S[ci] = dot / a^T a (the E or E^T correction), 0 once done.
__global__ __launch_bounds__(256) void k_sc_fl_ecoef(double *S, const double *p, int64_t n, int ci)
{
    __shared__ double red[4];
    const double d = sum_parts(p, n, red);
    if (threadIdx.x != 0) return;
    const double ca = S[S_FL_CA];
    const double c = (S[S_DONE] == 0.0 && ca > 0.0) ? d / ca : 0.0;
    S[ci] = finite(c) ? c : 0.0;
}

// Inner CG start from the sums of the right-hand side r: mu = mean(r),
// gamma = ||r - mu||^2.
__global__ __launch_bounds__(256) void k_sc_fl_cg_init(double *S, const double *ps, int64_t ns, const double *pq,
                                                       int64_t nq, int64_t n)
{
    __shared__ double red[4];
    const double s1 = sum_parts(ps, ns, red);
    const double s2 = sum_parts(pq, nq, red);
    if (threadIdx.x != 0) return;
    const double mu = s1 / double(n);
    const double g = s2 - double(n) * mu * mu;
    const bool ok = finite(mu) && finite(g);
    S[S_CG_MU] = ok ? mu : 0.0;
    S[S_CG_GAMMA] = ok ? fmax(g, 0.0) : 0.0;
    S[S_CG_BETA] = 0.0;
}

__global__ __launch_bounds__(256) void k_sc_fl_cg_alpha(double *S, const double *p, int64_t n)
{
    __shared__ double red[4];
    const double pq = sum_parts(p, n, red);
    if (threadIdx.x != 0) return;
    const double g = S[S_CG_GAMMA];
    const double a = (g > 0.0 && pq > 0.0) ? g / pq : 0.0;
    S[S_CG_ALPHA] = finite(a) ? a : 0.0;
}

__global__ __launch_bounds__(256) void k_sc_fl_cg_beta(double *S, const double *ps, int64_t ns, const double *pq,
                                                       int64_t nq, int64_t n)
{
    __shared__ double red[4];
    const double s1 = sum_parts(ps, ns, red);
    const double s2 = sum_parts(pq, nq, red);
    if (threadIdx.x != 0) return;
    const double mu = s1 / double(n);
    const double gn = fmax(s2 - double(n) * mu * mu, 0.0);
    const double g = S[S_CG_GAMMA];
    const bool ok = finite(mu) && finite(gn) && g > 0.0 && S[S_CG_ALPHA] > 0.0;
    S[S_CG_MU] = ok ? mu : 0.0;
    S[S_CG_BETA] = ok ? gn / g : 0.0;
    S[S_CG_GAMMA] = ok ? gn : 0.0;
}

// Norm of the new gradient-space vector: a zero norm means the flexible
// space cannot grow (done = 1); S_V0 = 1 / norm normalises it.
__global__ __launch_bounds__(256) void k_sc_fl_vnorm(double *S, const double *p, int64_t n)
{
    __shared__ double red[4];
    const double v2 = sum_parts(p, n, red);
    if (threadIdx.x != 0) return;
    const double t = sqrt(v2);
    S[S_V0] = 0.0;
    if (S[S_DONE] != 0.0) return;
    S[S_FL_TKK] = t;
    if (!finite(t)) S[S_DONE] = 2.0;
    else if (t == 0.0) S[S_DONE] = 1.0;
    else S[S_V0] = 1.0 / t;
}

// History row of iteration k: [(projected residual, set later), t_kk,
// M[k+1, k], done, (lambda_k, set later)]; advances the row counter.
__global__ void k_sc_fl_hist(double *S, const double *M, int k, int ldm, double *hist)
{
    if (threadIdx.x != 0) return;
    const int64_t row = int64_t(S[S_HROW]);
    if (hist && row < int64_t(S[S_ITER])) {
        double *h = hist + row * KCT_HIST_COLS;
        const bool live = int(S[S_KGK]) == k + 1;
        h[0] = 0.0;
        h[1] = live ? S[S_FL_TKK] : 0.0;
        h[2] = live ? M[int64_t(k) * ldm + k + 1] : 0.0;
        h[3] = hist_code(S);
        h[4] = S[S_HLAM];
    }
    S[S_HROW] = double(row + 1);
}

} // namespace

// A multiple of 8 workgroups (the XCD-aware row order needs it).
int fl_groups(int64_t n)
{
    const int64_t g = (n + 1023) / 1024;
    return int(std::max<int64_t>(8, std::min<int64_t>((g + 7) / 8 * 8, 2048)));
}

#define FL_CHECK(what) return check_hip(hipGetLastError(), what)

kct_status fl_lap(const Plan &p, const double *pv, const float *Lw, double *q, double *parts, hipStream_t st)
{
    const Dims d = dims(p);
    hipLaunchKernelGGL(k_fl_lap, dim3(fl_groups(d.M)), dim3(256), 0, st, pv, Lw, d, q, parts);
    FL_CHECK("weighted Laplacian");
}

kct_status fl_cg_update(double *t, double *r, const double *pv, const double *q, int64_t n, const double *S,
                        double *psum, double *psq, hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_cg_update, dim3(fl_groups(n)), dim3(256), 0, st, t, r, pv, q, n, S, psum, psq);
    FL_CHECK("inner CG update");
}

kct_status fl_cg_dir(double *r, double *pv, double *t, const float *rhs, int64_t n, const double *S, hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_cg_dir, dim3(fl_groups(n)), dim3(256), 0, st, r, pv, t, rhs, n, S);
    FL_CHECK("inner CG direction");
}

kct_status fl_to_f32(float *out, const double *in, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_to_f32, dim3(fl_groups(n)), dim3(256), 0, st, out, in, n);
    FL_CHECK("inner CG result");
}

kct_status fl_dtl(const Plan &p, const float *v3, const float *Lw, float *out, double *psum, double *psq,
                  hipStream_t st)
{
    const Dims d = dims(p);
    hipLaunchKernelGGL(k_fl_dtl, dim3(fl_groups(d.M)), dim3(256), 0, st, v3, Lw, d, out, psum, psq);
    FL_CHECK("weighted divergence");
}

kct_status fl_sum(const float *v, int64_t n, double *parts, hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_sum, dim3(fl_groups(n)), dim3(256), 0, st, v, n, parts);
    FL_CHECK("sum");
}

kct_status fl_axpy_sum(float *r, const float *g, int64_t n, const double *S, int ci, double *psum, double *psq,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_axpy_sum, dim3(fl_groups(n)), dim3(256), 0, st, r, g, n, S, ci, psum, psq);
    FL_CHECK("E^T correction");
}

kct_status fl_shift(float *out, const float *in, int64_t n, const double *S, int ci, hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_shift, dim3(fl_groups(n)), dim3(256), 0, st, out, in, n, S, ci);
    FL_CHECK("E correction");
}

kct_status fl_fill_s(float *out, int64_t n, const double *S, int ci, hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_fill_s, dim3(fl_groups(n)), dim3(256), 0, st, out, n, S, ci);
    FL_CHECK("fill");
}

kct_status fl_bbar(float *out, const float *b, const float *a, int64_t n, const double *S, double *parts,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_bbar, dim3(fl_groups(n)), dim3(256), 0, st, out, b, a, n, S, parts);
    FL_CHECK("bbar");
}

kct_status fl_combine(float *x, const float *Z, int64_t n, const double *coef, const double *S, hipStream_t st)
{
    hipLaunchKernelGGL(k_fl_combine, dim3(fl_groups(n)), dim3(256), 0, st, x, Z, n, coef, S);
    FL_CHECK("flexible combination");
}

kct_status fl_sc_init(double *S, Reduced ca, Reduced ab, int n_iter, double lam, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_init, dim3(1), dim3(256), 0, st, S, ca.ptr, ca.n, ab.ptr, ab.n, n_iter, lam);
    FL_CHECK("fLSQR init");
}

kct_status fl_sc_beta1(double *S, Reduced b2, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_beta1, dim3(1), dim3(256), 0, st, S, b2.ptr, b2.n);
    FL_CHECK("fLSQR beta1");
}

kct_status fl_sc_ecoef(double *S, Reduced dot, int ci, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_ecoef, dim3(1), dim3(256), 0, st, S, dot.ptr, dot.n, ci);
    FL_CHECK("E coefficient");
}

kct_status fl_sc_cg_init(double *S, Reduced sum, Reduced sq, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_cg_init, dim3(1), dim3(256), 0, st, S, sum.ptr, sum.n, sq.ptr, sq.n, n);
    FL_CHECK("inner CG init");
}

kct_status fl_sc_cg_alpha(double *S, Reduced pq, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_cg_alpha, dim3(1), dim3(256), 0, st, S, pq.ptr, pq.n);
    FL_CHECK("inner CG alpha");
}

kct_status fl_sc_cg_beta(double *S, Reduced sum, Reduced sq, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_cg_beta, dim3(1), dim3(256), 0, st, S, sum.ptr, sum.n, sq.ptr, sq.n, n);
    FL_CHECK("inner CG beta");
}

kct_status fl_sc_vnorm(double *S, Reduced v2, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_vnorm, dim3(1), dim3(256), 0, st, S, v2.ptr, v2.n);
    FL_CHECK("fLSQR vector norm");
}

kct_status fl_sc_hist(double *S, const double *M, int k, int ldm, double *hist, hipStream_t st)
{
    hipLaunchKernelGGL(k_sc_fl_hist, dim3(1), dim3(64), 0, st, S, M, k, ldm, hist);
    FL_CHECK("fLSQR history");
}

} // namespace kct
