// Unmatched back projection x = B y, gfx950: the voxel-driven interpolating
// back projector that GPU toolboxes use in place of A^T (paper Sec. 2.1.4);
// AB- and BA-GMRES take it as a right or left preconditioner.
//
// For voxel centre p and angle t (flat detector, circular orbit):
//   w = DSO - (p_x cos t + p_y sin t)       depth of p along the central ray
//   u = DSD (-p_x sin t + p_y cos t) / w,   v = DSD p_z / w
//   x_j += V / (du dv) (DSD / w)^2 |d| / DSD * bilinear(y_t, u, v)
// with |d| = sqrt(DSD^2 + u^2 + v^2), V the voxel volume, and the detector
// read as zero outside its pixel grid.  The weight makes B equal A^T for
// smooth data (rays cross the voxel at a density (DSD/w)^2 / (du dv cos g)
// per unit normal area, cos g = DSD / |d|).
//
// A thread owns one (i, j) voxel column and KZ voxels along z: w, u and the
// column's detector coordinate are computed once per angle (FP64), each voxel
// then costs one FP64 product for v, the bilinear weights (FP32) and four
// gathers.  Sums are FP32 per voxel, in angle order (deterministic).

#include "kct_internal.hpp"

#include <algorithm>

namespace kct {

namespace {

constexpr int IBP_TX = 16, IBP_TY = 16;

__device__ inline double block_sum_256i(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
    return s;
}

template <typename TP>
__device__ inline float tap(const TP *__restrict__ ya, int nu, int nv, int iu, int iv)
{
    return (iu >= 0 && iu < nu && iv >= 0 && iv < nv) ? to_f32(ya[int64_t(iv) * nu + iu]) : 0.f;
}

template <typename TP, typename TV, int KZ>
__global__ __launch_bounds__(256) void k_interp_bp(const TP *__restrict__ proj, TV *__restrict__ vol,
                                                   const AngleGeo *__restrict__ tab, GeoParams g, int tiles_x,
                                                   int tiles_y, int64_t groups, int64_t xcd_chunk, Epilogue ep)
{
    __shared__ double red[4];
    // The XCDs (b mod 8) take the tiles in turns of xcd_chunk consecutive
    // tiles (whole rows, as the matched back projector does), or one
    // contiguous eighth each when xcd_chunk <= 0.
    const int64_t g8 = (groups + 7) / 8;
    const int64_t b = blockIdx.x;
    const int64_t C = xcd_chunk > 0 ? xcd_chunk : g8;
    const int64_t k = b >> 3, q = k / C, r = k - q * C;
    const int64_t logical = q * 8 * C + (b & 7) * min(C, g8 - q * C) + r;
    if (logical >= groups) return;
    if (ep.scal && ep.scal[S_DONE] != 0.0) return;

    double c0 = ep.c[0], c1 = ep.c[1], c2 = ep.c[2], c3 = ep.c[3];
    if (ep.coef_idx >= 0) {
        c0 = ep.scal[ep.coef_idx];
        c1 = ep.scal[ep.coef_idx + 1];
        c2 = ep.scal[ep.coef_idx + 2];
        c3 = ep.scal[ep.coef_idx + 3];
    }
    const int per_z = tiles_x * tiles_y;
    const int tz = int(logical / per_z);
    const int rem = int(logical - int64_t(tz) * per_z);
    const int tyi = rem / tiles_x, txi = rem - tyi * tiles_x;
    const int i = txi * IBP_TX + (threadIdx.x & 15), j = tyi * IBP_TY + (threadIdx.x >> 4), k0 = tz * KZ;
    const bool valid = i < g.nx && j < g.ny;

    float acc[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) acc[kk] = 0.f;

    if (valid) {
        const double x = g.X0 + (i + 0.5) * g.vx, y = g.Y0 + (j + 0.5) * g.vy;
        const double wvol = g.vx * g.vy * g.vz / (g.du * g.dv);
        const double idu = 1.0 / g.du, idv = 1.0 / g.dv;
        for (int a = 0; a < g.na; ++a) {
            const AngleGeo A = tab[a];
            const double w = g.dso - (x * A.cs + y * A.sn);
            const double rw = g.dsd / w;
            const double u = (-x * A.sn + y * A.cs) * rw;
            const double fu = u * idu + g.cu;
            const double fl = floor(fu);
            const int iu0 = int(fl);
            const float au = float(fu - fl);
            const float wb = float(wvol * rw * rw / g.dsd);
            const float u2d2 = float(g.dsd * g.dsd + u * u);
            const TP *ya = proj + int64_t(a) * g.nv * g.nu;
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const int k = k0 + kk;
                if (k < g.nz) {
                    const double v = (g.Z0 + (k + 0.5) * g.vz) * rw;
                    const double fv = v * idv + g.cv;
                    const double flv = floor(fv);
                    const int iv0 = int(flv);
                    const float av = float(fv - flv);
                    const float t00 = tap(ya, g.nu, g.nv, iu0, iv0), t01 = tap(ya, g.nu, g.nv, iu0 + 1, iv0);
                    const float t10 = tap(ya, g.nu, g.nv, iu0, iv0 + 1), t11 = tap(ya, g.nu, g.nv, iu0 + 1, iv0 + 1);
                    const float val = (1.f - av) * ((1.f - au) * t00 + au * t01) + av * ((1.f - au) * t10 + au * t11);
                    const float dn = sqrtf(u2d2 + float(v * v));
                    acc[kk] = fmaf(wb * dn, val, acc[kk]);
                }
            }
        }
    }

    double part = 0.0;
    if (valid) {
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            const int k = k0 + kk;
            if (k < g.nz) {
                const int64_t idx = (int64_t(k) * g.ny + j) * g.nx + i;
                double o = c0 * double(acc[kk]);
                if (ep.in1 && c1 != 0.0) o += c1 * double(to_f32(static_cast<const TV *>(ep.in1)[idx]));
                if (ep.in2 && c2 != 0.0) o += c2 * double(ep.in2[idx]);
                if (ep.in3 && c3 != 0.0) o += c3 * double(to_f32(static_cast<const TV *>(ep.in3)[idx]));
                const TV st = from_f32<TV>(float(o));
                vol[idx] = st;
                const double sv = double(to_f32(st));
                part += sv * sv;
            }
        }
    }
    if (ep.partials) {
        const double s = block_sum_256i(part, red);
        if (threadIdx.x == 0) ep.partials[logical] = s;
    }
}

constexpr int IBP_KZ = 8;

template <typename TP, typename TV>
kct_status ibp_launch(Plan &p, const void *proj, void *vol, const Epilogue &ep, hipStream_t st)
{
    const int64_t tiles_x = (p.gp.nx + IBP_TX - 1) / IBP_TX, tiles_y = (p.gp.ny + IBP_TY - 1) / IBP_TY;
    const int64_t groups = tiles_x * tiles_y * ((p.gp.nz + IBP_KZ - 1) / IBP_KZ);
    const int64_t launch = ((groups + 7) / 8) * 8;
    if (launch * 256 >= (int64_t(1) << 32)) return fail(KCT_E_GEOMETRY, "interpolating back projection grid too large");
    hipLaunchKernelGGL((k_interp_bp<TP, TV, IBP_KZ>), dim3(unsigned(launch)), dim3(256), 0, st,
                       static_cast<const TP *>(proj), static_cast<TV *>(vol), p.d_tab, p.gp, int(tiles_x),
                       int(tiles_y), groups, p.bwd_xcd_chunk, ep);
    return check_hip(hipGetLastError(), "interpolating back projection launch");
}

} // namespace

int64_t ibp_num_groups(const Plan &p)
{
    const int64_t tiles_x = (p.gp.nx + IBP_TX - 1) / IBP_TX, tiles_y = (p.gp.ny + IBP_TY - 1) / IBP_TY;
    return tiles_x * tiles_y * ((p.gp.nz + IBP_KZ - 1) / IBP_KZ);
}

kct_status launch_interp_backward(Plan &p, const void *proj, int proj_dtype, void *vol, int vol_dtype,
                                  const Epilogue &ep, hipStream_t st)
{
    if (proj_dtype == KCT_F32 && vol_dtype == KCT_F32) return ibp_launch<float, float>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_BF16 && vol_dtype == KCT_BF16) return ibp_launch<bf16, bf16>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F16 && vol_dtype == KCT_F16) return ibp_launch<_Float16, _Float16>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_BF16 && vol_dtype == KCT_F32) return ibp_launch<bf16, float>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F16 && vol_dtype == KCT_F32) return ibp_launch<_Float16, float>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F32 && vol_dtype == KCT_BF16) return ibp_launch<float, bf16>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F32 && vol_dtype == KCT_F16) return ibp_launch<float, _Float16>(p, proj, vol, ep, st);
    return fail(KCT_E_DTYPE, "unsupported storage pair for the interpolating back projector");
}

} // namespace kct
