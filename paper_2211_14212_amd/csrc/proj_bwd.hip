// Matched back projection x = A^T y, gfx950.
//
// Exact transpose of the forward projector: x_j = sum_i a_ij y_i with the
// same a_ij = length (mm) of ray i inside voxel j.  The forward kernel walks
// rays; this kernel gathers per voxel, so no atomics and a fixed summation
// order (bitwise reproducible).  For voxel j and angle t it enumerates the
// pixels whose centres fall inside the perspective footprint of the voxel (the
// box spanned by its projected corners, which contains the projection of the
// whole convex voxel) and intersects each pixel's ray with the voxel's three
// slabs in FP64:
//     t in [(x0-sx)/dx, (x1-sx)/dx] n [(y0-sy)/dy, ...] n [z0/v, z1/v],
// length = (t_hi - t_lo)+ * |d|.  Rays whose centre lies outside the footprint
// meet the voxel in at most a point, so the sum equals the forward
// projector's row-wise sum up to rounding.
//
// Structure (flat circular detector, e_v = z): the x/y slab interval of a ray
// depends only on its detector column u, the z interval only on its row v.  A
// thread owns one (i, j) voxel column and KZ voxels along z, so the per-column
// x/y intervals are computed once per angle and reused by its KZ voxels; each
// candidate pixel then costs a max, a min, a subtraction and one FMA with the
// staged value.  A workgroup is a 16 x 16 x KZ voxel tile; per angle it stages
// the tile's detector footprint (values pre-multiplied by the ray length |d|)
// and the per-column 1/dx, 1/dy and per-row 1/v in LDS.
//
// Sparse rays (k_backward_rays).  When the detector samples the volume more
// coarsely than the voxel grid (micro-CT: 0.37 nonzeros per voxel-view), most
// voxel-views hold no nonzero and the per-voxel candidate search above costs
// far more than the sums.  If every voxel's footprint is narrower than one
// pixel along u and along v (checked on the host from the extreme
// magnification), at most one ray of an angle meets any voxel.  The kernel
// then walks rays instead: a workgroup owns a 16 x 16 x 8 voxel tile with its
// sums in LDS, and its lanes trace the rays of the tile's footprint through
// the tile, adding length * value to the voxels they cross.  Rays of one
// angle never share a voxel, so a lane's read-add-write of a voxel sum meets
// no other lane's.  Up to four consecutive angles run side by side, each
// into its own copy of the tile sums, and a barrier separates these passes,
// so every sum receives its terms in a fixed order (angle order within a
// copy, then the four copies added in order): the result is deterministic
// and needs no atomics.  Lengths come from the same FP64 slab-crossing walk
// as the forward projector's.

#include "kct_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

namespace kct {

namespace {

constexpr int BWD_TX = 16, BWD_TY = 16;

__device__ inline double block_sum_256b(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((red[0] + red[1]) + red[2]) + red[3];
    return s;
}

__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Detector footprint of the tile at one angle: [iu_lo, iu_hi] x [iv_lo, iv_hi]
// (empty when hi < lo).  FP32 with fast reciprocals: the bounds only select
// candidate pixels, widened by `margin`; the FP64 intervals decide lengths.
struct Footprint {
    int iu_lo, iu_hi, iv_lo, iv_hi;
};

__device__ inline Footprint tile_footprint(const AngleGeo &A, const GeoParams &g, float tx0, float tx1, float ty0,
                                           float ty1, float tz0, float tz1, float margin)
{
    const float cs = float(A.cs), sn = float(A.sn), dsd = float(g.dsd), dso = float(g.dso);
    const float idu = float(1.0 / g.du), idv = float(1.0 / g.dv), cu = float(g.cu), cv = float(g.cv);
    float umin = 3.0e38f, umax = -3.0e38f, wmin = 3.0e38f, wmax = -3.0e38f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float x = (q & 1) ? tx1 : tx0, y = (q & 2) ? ty1 : ty0;
        const float w = dso - (x * cs + y * sn);
        const float u = dsd * (-x * sn + y * cs) * fast_rcp(w);
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        wmin = fminf(wmin, w);
        wmax = fmaxf(wmax, w);
    }
    const float ra = dsd * fast_rcp(wmin), rb = dsd * fast_rcp(wmax);
    const float va = tz0 * ra, vb = tz0 * rb, vc = tz1 * ra, vd = tz1 * rb;
    const float vmin = fminf(fminf(va, vb), fminf(vc, vd)), vmax = fmaxf(fmaxf(va, vb), fmaxf(vc, vd));
    Footprint f;
    f.iu_lo = max(0, int(ceilf(umin * idu + cu - margin)));
    f.iu_hi = min(g.nu - 1, int(floorf(umax * idu + cu + margin)));
    f.iv_lo = max(0, int(ceilf(vmin * idv + cv - margin)));
    f.iv_hi = min(g.nv - 1, int(floorf(vmax * idv + cv + margin)));
    return f;
}

// |pixel centre - source| per detector pixel (angle-independent), the
// factor the back projector applies to every staged value.
__global__ __launch_bounds__(256) void k_ray_lengths(float *__restrict__ out, GeoParams g)
{
    const int64_t n = int64_t(g.nu) * g.nv;
    const float dsd = float(g.dsd);
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
        const int iv = int(e / g.nu), iu = int(e - int64_t(iv) * g.nu);
        const float uu = float((iu - g.cu) * g.du), vv = float((iv - g.cv) * g.dv);
        out[e] = sqrtf(dsd * dsd + uu * uu + vv * vv);
    }
}

// Tile of workgroup b.  The workgroups of one dispatch go to the 8 XCDs in
// turn (b mod 8); XCD x's k-th workgroup (k = b / 8) takes chunk q = k / C of
// C consecutive tiles: tiles q * 8C + x * w + k mod C, w = min(C, g8 - q * C)
// (a bijection onto [0, 8 * g8)).  C = g8 (xcd_chunk <= 0) gives each XCD one
// contiguous eighth of the tiles; C = one row of tiles keeps the 8 XCDs on
// neighbouring rows of one z-layer, whose footprints overlap in the MALL.
__device__ inline int64_t bwd_logical_tile(int64_t b, int64_t groups, int64_t xcd_chunk)
{
    const int64_t g8 = (groups + 7) / 8;
    const int64_t C = xcd_chunk > 0 ? xcd_chunk : g8;
    const int64_t k = b >> 3, q = k / C, r = k - q * C;
    return q * 8 * C + (b & 7) * min(C, g8 - q * C) + r;
}

template <typename TP, typename TV, int KZ, int NCM, bool ACC_LDS>
__global__ __launch_bounds__(256) void k_backward(const TP *__restrict__ proj, TV *__restrict__ vol,
                                                  const AngleGeo *__restrict__ tab,
                                                  const double *__restrict__ invv,
                                                  const float *__restrict__ dlen, GeoParams g, int tiles_x,
                                                  int tiles_y, int64_t groups, int pw_max, int ph_max,
                                                  int fp_angles, int *err_flag, int64_t xcd_chunk, Epilogue ep)
{
    // Angle chunk of this workgroup: all angles, or (small volumes) chunk
    // blockIdx.y of gridDim.y, whose raw sums go to the partial volumes.
    const int chunks = int(gridDim.y), chunk = int(blockIdx.y);
    const int a_begin = int(int64_t(g.na) * chunk / chunks), a_end = int(int64_t(g.na) * (chunk + 1) / chunks);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double *cinv = reinterpret_cast<double *>(lds_raw);       // 2 * pw_max
    double *rinv = cinv + 2 * pw_max;                         // ph_max
    int4 *fps = reinterpret_cast<int4 *>(rinv + ph_max);      // fp_angles tile footprints
    float *accs = reinterpret_cast<float *>(fps + fp_angles);  // KZ * 256 when ACC_LDS
    float *patch = accs + (ACC_LDS ? KZ * 256 : 0);            // pw_max * ph_max + NCM
    __shared__ double red[4];

    const int64_t logical = bwd_logical_tile(blockIdx.x, groups, xcd_chunk);
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
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int i = txi * BWD_TX + lx, j = tyi * BWD_TY + ly, k0 = tz * KZ;
    const bool valid = i < g.nx && j < g.ny;

    const double x0 = g.X0 + i * g.vx, x1 = x0 + g.vx;
    const double y0 = g.Y0 + j * g.vy, y1 = y0 + g.vy;
    const int ie = min(txi * BWD_TX + BWD_TX, g.nx), je = min(tyi * BWD_TY + BWD_TY, g.ny);
    const int ke = min(k0 + KZ, g.nz);
    const float tx0 = float(g.X0 + txi * BWD_TX * g.vx), tx1 = float(g.X0 + ie * g.vx);
    const float ty0 = float(g.Y0 + tyi * BWD_TY * g.vy), ty1 = float(g.Y0 + je * g.vy);
    const float tz0 = float(g.Z0 + k0 * g.vz), tz1 = float(g.Z0 + ke * g.vz);
    const float dsd = float(g.dsd), dso = float(g.dso);
    const float idu = float(1.0 / g.du), idv = float(1.0 / g.dv), cu = float(g.cu), cv = float(g.cv);
    const float margin = 0.01f; // pixels; the exact FP64 intervals reject extra candidates

    // Tile footprints of every angle (or of the first fp_angles), computed once.
    for (int a = a_begin + threadIdx.x; a < min(a_end, fp_angles); a += 256) {
        const Footprint f = tile_footprint(tab[a], g, tx0, tx1, ty0, ty1, tz0, tz1, margin);
        fps[a] = make_int4(f.iu_lo, f.iu_hi, f.iv_lo, f.iv_hi);
    }
    __syncthreads();

    // Per-voxel sums: registers (fully unrolled z run) or this thread's LDS
    // slots (rolled loop, fewer registers).
    float acc[ACC_LDS ? 1 : KZ];
#pragma unroll
    for (int kk = 0; kk < (ACC_LDS ? 1 : KZ); ++kk) acc[kk] = 0.f;
    if constexpr (ACC_LDS)
        for (int kk = 0; kk < KZ; ++kk) accs[kk * 256 + threadIdx.x] = 0.f;

    for (int a = a_begin; a < a_end; ++a) {
        const AngleGeo A = tab[a];
        Footprint f;
        if (a < fp_angles) {
            const int4 q = fps[a];
            f = Footprint{q.x, q.y, q.z, q.w};
        } else {
            f = tile_footprint(A, g, tx0, tx1, ty0, ty1, tz0, tz1, margin);
        }
        const int iu_lo = f.iu_lo, iu_hi = f.iu_hi, iv_lo = f.iv_lo;
        int pw = iu_hi - iu_lo + 1, ph = f.iv_hi - iv_lo + 1;
        if (pw <= 0 || ph <= 0) continue;
        if (pw > pw_max || ph > ph_max) {
            // Never expected (the plan's bounds come from the extreme
            // magnification): the sums are truncated, and the caller learns
            // it from kct_plan_check or history code 4.
            if (threadIdx.x == 0) {
                if (err_flag) atomicOr(err_flag, 1);
                if (ep.err_scal) ep.err_scal[S_ERR] = 1.0;
            }
            pw = min(pw, pw_max);
            ph = min(ph, ph_max);
        }

        __syncthreads(); // the previous angle's reads of LDS are done
        const TP *ya = proj + int64_t(a) * g.nv * g.nu;
        {
            // Patch element e = r * pw + c, walked without a division per
            // element: each step of 256 advances (r, c) by (q, rem).
            const int q = 256 / pw, rem = 256 - q * pw;
            int r = threadIdx.x / pw, c = threadIdx.x - (threadIdx.x / pw) * pw;
#pragma unroll 4
            for (int e = threadIdx.x; e < pw * ph; e += 256) {
                const int64_t pix = int64_t(iv_lo + r) * g.nu + (iu_lo + c);
                patch[e] = to_f32(ya[pix]) * dlen[pix];
                c += rem;
                r += q;
                if (c >= pw) {
                    c -= pw;
                    ++r;
                }
            }
        }
        for (int c = threadIdx.x; c < pw; c += 256) {
            // 1/d per axis; 0 marks a ray parallel to that axis's planes.
            const double u = (iu_lo + c - g.cu) * g.du;
            const double dxm = -g.dsd * A.cs - u * A.sn, dym = -g.dsd * A.sn + u * A.cs;
            cinv[2 * c] = dxm != 0.0 ? 1.0 / dxm : 0.0;
            cinv[2 * c + 1] = dym != 0.0 ? 1.0 / dym : 0.0;
        }
        for (int r = threadIdx.x; r < ph; r += 256) rinv[r] = invv[iv_lo + r];
        // The unrolled column loop reads up to NCM-1 values past the patch;
        // they are multiplied by a zero length, so they must be finite.
        if (threadIdx.x < NCM) patch[pw * ph + threadIdx.x] = 0.f;
        __syncthreads();

        if (valid) {
            const float cs = float(A.cs), sn = float(A.sn);
            // Own column footprint.
            float cumin = 3.0e38f, cumax = -3.0e38f, cwmin = 3.0e38f, cwmax = -3.0e38f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float x = float((q & 1) ? x1 : x0), y = float((q & 2) ? y1 : y0);
                const float w = dso - (x * cs + y * sn);
                const float u = dsd * (-x * sn + y * cs) * fast_rcp(w);
                cumin = fminf(cumin, u);
                cumax = fmaxf(cumax, u);
                cwmin = fminf(cwmin, w);
                cwmax = fmaxf(cwmax, w);
            }
            const int c_lo = max(iu_lo, int(ceilf(cumin * idu + cu - margin)));
            int nc = min(iu_hi, int(floorf(cumax * idu + cu + margin))) - c_lo + 1;
            if (nc > NCM) { // never expected either; reported like the patch overflow
                if (err_flag) atomicOr(err_flag, 2);
                if (ep.err_scal) ep.err_scal[S_ERR] = 1.0;
                nc = NCM;
            }
            nc = min(nc, pw - (c_lo - iu_lo)); // stay inside the staged patch
            // Columns any lane of the wave needs: the unrolled candidate loop
            // skips the rest with a scalar branch.
            int ncw = 1;
#pragma unroll
            for (int c = 1; c < NCM; ++c)
                if (__any(nc > c)) ncw = c + 1;
            const double ax0 = x0 - A.sx, ax1 = x1 - A.sx, ay0 = y0 - A.sy, ay1 = y1 - A.sy;
            constexpr double FAR = 1.0e300;
            double lo[NCM], hi[NCM];
#pragma unroll
            for (int c = 0; c < NCM; ++c) {
                lo[c] = 1.0;
                hi[c] = 0.0;
                if (c < nc) {
                    const int ci = c_lo - iu_lo + c;
                    const double ix = cinv[2 * ci], iy = cinv[2 * ci + 1];
                    double xl, xh, yl, yh;
                    if (ix != 0.0) {
                        const double ta = ax0 * ix, tb = ax1 * ix;
                        xl = fmin(ta, tb);
                        xh = fmax(ta, tb);
                    } else { // parallel to x-planes: inside iff x0 <= sx < x1
                        const bool in = ax0 <= 0.0 && 0.0 < ax1;
                        xl = in ? -FAR : FAR;
                        xh = in ? FAR : -FAR;
                    }
                    if (iy != 0.0) {
                        const double tc = ay0 * iy, td = ay1 * iy;
                        yl = fmin(tc, td);
                        yh = fmax(tc, td);
                    } else {
                        const bool in = ay0 <= 0.0 && 0.0 < ay1;
                        yl = in ? -FAR : FAR;
                        yh = in ? FAR : -FAR;
                    }
                    lo[c] = fmax(xl, yl);
                    hi[c] = fmin(xh, yh);
                }
            }
            const float *pcol = patch + (c_lo - iu_lo);
            // Detector rows per mm of z at the column's nearest and farthest
            // corner from the source (both magnifications are positive).
            const float ra = dsd * fast_rcp(cwmin) * idv, rb = dsd * fast_rcp(cwmax) * idv;
            const float rhi = fmaxf(ra, rb), rlo = fminf(ra, rb);
            const float cvp = cv + margin, cvm = cv - margin;
            const int r_end = iv_lo + ph - 1;
            // The z run, compiled for the wave's column count NC <= NCM.  Row
            // bounds come from the z-planes of the thread's voxels: voxel k
            // spans rows [row_lo(z_k), row_hi(z_{k+1})], where a plane at
            // height z projects between rows cv + z * rlo and cv + z * rhi
            // (ordered by the sign of z).  FP32 is enough: the bounds only
            // select candidate rows, with a margin far above their rounding.
            auto zrun = [&](auto nct) {
                constexpr int NC = decltype(nct)::value;
                const float zb = float(g.Z0 + k0 * g.vz), vzf = float(g.vz);
                float lo_b = fmaf(zb, zb >= 0.f ? rlo : rhi, cvm);
#pragma unroll(ACC_LDS ? 1 : KZ)
                for (int kk = 0; kk < KZ; ++kk) {
                    const int k = k0 + kk;
                    const float zt = fmaf(float(kk + 1), vzf, zb);
                    const bool up = zt >= 0.f;
                    const float hi_t = fmaf(zt, up ? rhi : rlo, cvp);
                    const float lo_t = fmaf(zt, up ? rlo : rhi, cvm);
                    if (k < g.nz && nc > 0) {
                        const double z0 = g.Z0 + k * g.vz, z1 = z0 + g.vz;
                        const int r_lo = max(iv_lo, int(ceilf(lo_b)));
                        const int r_hi = min(r_end, int(floorf(hi_t)));
                        float s = ACC_LDS ? accs[kk * 256 + threadIdx.x] : acc[ACC_LDS ? 0 : kk];
                        for (int r = r_lo; r <= r_hi; ++r) {
                            // 1/v of the row (a huge positive value for v = 0, which
                            // keeps the half-open rule: z0 <= 0 < z1 gives an
                            // interval covering every t in (0, 1)).
                            const double iv = rinv[r - iv_lo];
                            const double ta = z0 * iv, tb = z1 * iv;
                            const double zl = fmin(ta, tb), zh = fmax(ta, tb);
                            const float *prow = pcol + (r - iv_lo) * pw;
#pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                const double len = fmin(hi[c], zh) - fmax(lo[c], zl);
                                // Clamping to [0, 1] (an interval inside one voxel
                                // is far shorter than the whole ray) folds into
                                // the subtraction's clamp bit.
                                s = fmaf(float(fmin(fmax(len, 0.0), 1.0)), prow[c], s);
                            }
                        }
                        if constexpr (ACC_LDS) accs[kk * 256 + threadIdx.x] = s;
                        else acc[ACC_LDS ? 0 : kk] = s;
                    }
                    lo_b = lo_t;
                }
            };
            if (NCM >= 2 && ncw <= 2) zrun(std::integral_constant<int, (NCM >= 2 ? 2 : NCM)>{});
            else if (NCM >= 3 && ncw <= 3) zrun(std::integral_constant<int, (NCM >= 3 ? 3 : NCM)>{});
            else if (NCM >= 4 && ncw <= 4) zrun(std::integral_constant<int, (NCM >= 4 ? 4 : NCM)>{});
            else if (NCM >= 8 && ncw <= 8) zrun(std::integral_constant<int, (NCM >= 8 ? 8 : NCM)>{});
            else zrun(std::integral_constant<int, NCM>{});
        }
    }

    if (chunks > 1) { // raw sums of this chunk's angles; k_bwd_combine finishes
        if (valid) {
            float *dst = ep.split + int64_t(chunk) * g.nx * g.ny * g.nz;
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const int k = k0 + kk;
                if (k < g.nz)
                    dst[(int64_t(k) * g.ny + j) * g.nx + i] = ACC_LDS ? accs[kk * 256 + threadIdx.x]
                                                                     : acc[ACC_LDS ? 0 : kk];
            }
        }
        return;
    }
    double part = 0.0;
    if (valid) {
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            const int k = k0 + kk;
            if (k < g.nz) {
                const int64_t idx = (int64_t(k) * g.ny + j) * g.nx + i;
                const float a_k = ACC_LDS ? accs[kk * 256 + threadIdx.x] : acc[ACC_LDS ? 0 : kk];
                double o = c0 * double(a_k);
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
        const double s = block_sum_256b(part, red);
        if (threadIdx.x == 0) ep.partials[logical] = s;
    }
}

// ---------------------------------------------------------------------------
// Ray-driven back projection for sparse rays (see the top of this file).
// ---------------------------------------------------------------------------
constexpr int BR_TX = 16, BR_TY = 16, BR_TZ = 8;     // voxel tile
constexpr int BR_VOX = BR_TX * BR_TY * BR_TZ;        // 2048 sums per copy
// LDS layout of a copy: z-layers 257 floats apart and copies 2064 floats
// apart (16 banks apart).  Rays that walk in lockstep through the same
// (i, j) cells meet them at other z-layers (neighbouring detector rows) or
// in other copies (neighbouring angles); with a 256-float layer stride all
// of those sums would sit in one LDS bank and every read and write of the
// wave would serialise on it.
constexpr int BR_KS = BR_TX * BR_TY + 1;              // z-layer stride
constexpr int BR_CS = BR_TZ * BR_KS + 8;              // copy stride (2064)
constexpr int BR_LAST = (BR_TZ - 1) * BR_KS + BR_TX * BR_TY - 1; // last cell of a copy
constexpr int BR_COPIES = 4;                         // angles side by side
constexpr int BR_FP = 64;                            // tile footprints kept in LDS at a time
// Segments shorter than this (in units of the whole source-pixel ray) are
// skipped.  The walk's crossings carry ~1e-15 rounding; where a crossing
// rounds to just before the tile's exit, the walk takes one extra step out of
// the tile, onto a segment no longer than that rounding, which must not be
// written.  A real segment this short weighs 1e-12 of a ray (~1e-9 mm).
constexpr double BR_MIN_LEN = 1.0e-12;

// 0.0 or 1.0 from a predicate, built from the high word only (one select).
__device__ inline double br_one_if(bool c)
{
    return __builtin_bit_cast(double, uint64_t(c ? 0x3ff00000u : 0u) << 32);
}

template <typename TP, typename TV>
__global__ __launch_bounds__(256) void k_backward_rays(const TP *__restrict__ proj, TV *__restrict__ vol,
                                                       const AngleGeo *__restrict__ tab,
                                                       const double *__restrict__ invv,
                                                       const float *__restrict__ dlen, GeoParams g, int tiles_x,
                                                       int tiles_y, int64_t groups, int64_t xcd_chunk, Epilogue ep)
{
    const int chunks = int(gridDim.y), chunk = int(blockIdx.y);
    const int a_begin = int(int64_t(g.na) * chunk / chunks), a_end = int(int64_t(g.na) * (chunk + 1) / chunks);
    __shared__ float sums[BR_COPIES][BR_CS];
    __shared__ float junk_cell[1]; // sink of the walk's skipped segments (never read back)
    __shared__ int4 fps[BR_FP];
    __shared__ double red[4];

    const int64_t logical = bwd_logical_tile(blockIdx.x, groups, xcd_chunk);
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
    const int i0 = txi * BR_TX, j0 = tyi * BR_TY, k0 = tz * BR_TZ;
    const int ie = min(i0 + BR_TX, g.nx), je = min(j0 + BR_TY, g.ny), ke = min(k0 + BR_TZ, g.nz);
    const float tx0 = float(g.X0 + i0 * g.vx), tx1 = float(g.X0 + ie * g.vx);
    const float ty0 = float(g.Y0 + j0 * g.vy), ty1 = float(g.Y0 + je * g.vy);
    const float tz0 = float(g.Z0 + k0 * g.vz), tz1 = float(g.Z0 + ke * g.vz);
    const float margin = 0.01f; // pixels: the footprint only enumerates candidate rays

    for (int e = threadIdx.x; e < BR_COPIES * BR_CS; e += 256) (&sums[0][0])[e] = 0.f;

    unsigned pass = 0;
    for (int cb = a_begin; cb < a_end; cb += BR_FP) {
        const int ce = min(cb + BR_FP, a_end);
        __syncthreads(); // the previous chunk's footprints are no longer read
        if (threadIdx.x < ce - cb) {
            const Footprint f = tile_footprint(tab[cb + threadIdx.x], g, tx0, tx1, ty0, ty1, tz0, tz1, margin);
            fps[threadIdx.x] = make_int4(f.iu_lo, f.iu_hi, f.iv_lo, f.iv_hi);
        }
        __syncthreads();
        for (int a = cb; a < ce;) {
            // Pack up to BR_COPIES consecutive angles, m of them, such that m
            // times the largest footprint is at most 256 rays (a larger single
            // footprint takes a pass of its own, in rounds of 256).  Uniform
            // over the workgroup.
            int m = 0, nmax = 0;
#pragma unroll
            for (int q = 0; q < BR_COPIES; ++q) {
                if (a + q >= ce) break;
                const int4 f = fps[a + q - cb];
                const int n = max(0, f.y - f.x + 1) * max(0, f.w - f.z + 1);
                if (q > 0 && (q + 1) * max(nmax, n) > 256) break;
                nmax = max(nmax, n);
                m = q + 1;
            }
            // Lane t takes ray e = t / m of angle a + t mod m, so that each
            // wave holds the same ranks of all the pass's angles.  Within an
            // angle the rays are ranked by column, from the footprint's middle
            // column outwards (middle, right, left, ...), and by row within a
            // column.  A ray's path through the tile is longest at the middle
            // and shortens towards the edges, so a wave's lanes walk paths of
            // similar length and fewer of them idle while the longest one
            // finishes.
            // The wave that takes the middle (longest) ranks rotates from pass
            // to pass and between workgroups, so that the longest walks do
            // not always fall on the same SIMD of a CU.
            const float inv_m = __builtin_amdgcn_rcpf(float(m));
            const int lane_pos = (threadIdx.x + 64 * int((pass + blockIdx.x) & 3)) & 255;
            ++pass;
            for (int t = lane_pos; t < m * nmax; t += 256) {
                const int e = int((float(t) + 0.5f) * inv_m);
                const int q = t - e * m;
                const int aa = a + q;
                const int4 f = fps[aa - cb];
                const int pw = f.y - f.x + 1, ph = f.w - f.z + 1;
                if (pw <= 0 || ph <= 0 || e >= pw * ph) continue;
                const int rank = int((float(e) + 0.5f) * __builtin_amdgcn_rcpf(float(ph)));
                const int row = e - rank * ph;
                const int col = (pw - 1) / 2 + ((rank & 1) ? (rank + 1) >> 1 : -(rank >> 1));
                const int iu = f.x + col, iv = f.z + row;
                const int64_t pix = int64_t(iv) * g.nu + iu;
                const float yv = to_f32(proj[int64_t(aa) * g.nv * g.nu + pix]) * dlen[pix];
                if (yv == 0.f) continue;
                float *acc = sums[(aa - a_begin) % BR_COPIES];
                float *junk = junk_cell;

                // The ray from the source to the pixel centre, in the voxel
                // frame (voxel (i,j,k) = [i,i+1) x [j,j+1) x [k,k+1)), clipped
                // to the tile.
                const AngleGeo A = tab[aa];
                const double u = (iu - g.cu) * g.du, v = (iv - g.cv) * g.dv;
                const double dx = A.d0x + u * A.eux, dy = A.d0y + u * A.euy, dz = v * g.ivz;
                double tmin = 0.0, tmax = 1.0, inx = 0.0, iny = 0.0, inz = 0.0;
                if (dx != 0.0) {
                    inx = 1.0 / dx;
                    const double ta = (double(i0) - A.svx) * inx, tb = (double(ie) - A.svx) * inx;
                    tmin = fmax(tmin, fmin(ta, tb));
                    tmax = fmin(tmax, fmax(ta, tb));
                } else if (!(A.svx >= i0 && A.svx < ie)) {
                    continue;
                }
                if (dy != 0.0) {
                    iny = 1.0 / dy;
                    const double ta = (double(j0) - A.svy) * iny, tb = (double(je) - A.svy) * iny;
                    tmin = fmax(tmin, fmin(ta, tb));
                    tmax = fmin(tmax, fmax(ta, tb));
                } else if (!(A.svy >= j0 && A.svy < je)) {
                    continue;
                }
                if (dz != 0.0) {
                    // 1/dz = vz / v (the per-row table holds 1/v).
                    inz = g.vz * invv[iv];
                    const double ta = (double(k0) - A.svz) * inz, tb = (double(ke) - A.svz) * inz;
                    tmin = fmax(tmin, fmin(ta, tb));
                    tmax = fmin(tmax, fmax(ta, tb));
                } else if (!(A.svz >= k0 && A.svz < ke)) {
                    continue;
                }
                if (!(tmin < tmax)) continue;
                const int i = min(max(int(floor(A.svx + tmin * dx)), i0), ie - 1);
                const int j = min(max(int(floor(A.svy + tmin * dy)), j0), je - 1);
                const int k = min(max(int(floor(A.svz + tmin * dz)), k0), ke - 1);
                constexpr double FAR = 1.0e300;
                double txc = FAR, tyc = FAR, tzc = FAR, dtx = 0.0, dty = 0.0, dtz = 0.0;
                int sx = 0, sy = 0, sz = 0;
                if (dx > 0.0) { txc = (i + 1 - A.svx) * inx; dtx = inx; sx = 1; }
                else if (dx < 0.0) { txc = (i - A.svx) * inx; dtx = -inx; sx = -1; }
                if (dy > 0.0) { tyc = (j + 1 - A.svy) * iny; dty = iny; sy = BR_TX; }
                else if (dy < 0.0) { tyc = (j - A.svy) * iny; dty = -iny; sy = -BR_TX; }
                if (dz > 0.0) { tzc = (k + 1 - A.svz) * inz; dtz = inz; sz = BR_KS; }
                else if (dz < 0.0) { tzc = (k - A.svz) * inz; dtz = -inz; sz = -BR_KS; }
                int off = (k - k0) * BR_KS + (j - j0) * BR_TX + (i - i0);
                double tc = tmin;
                // Each step ends the current segment at the first crossing
                // (or the exit) and advances exactly one axis, x before y
                // before z on ties (a tie leaves a zero-length segment in a
                // diagonal neighbour).  While t < tmax the walk stays inside
                // the tile; at most nx+ny+nz+3 steps.  The sum of the next
                // voxel is read before the current one is written (they are
                // different voxels), so the read's latency overlaps a whole
                // step.  Segments no longer than BR_MIN_LEN (ties, and the
                // rounding-level step out of the tile at the exit) are
                // written to a scratch cell instead, and a read index outside
                // the tile is clamped into it (its value is then unused).
                // Two segments per trip, so that each read has a register of
                // its own and the loop carries no copy that would wait for it.
#define KCT_BR_STEP(CUR, NEXT)                                                                             \
    {                                                                                                      \
        const double m1 = fmin(txc, tyc);                                                                  \
        const double t1 = fmin(m1, tzc);                                                                   \
        const bool xy = txc <= tyc, first = m1 <= tzc;                                                     \
        float *dst = acc + off;                                                                            \
        off += first ? (xy ? sx : sy) : sz;                                                                \
        NEXT = acc[min(max(off, 0), BR_LAST)];                                                             \
        txc = fma(br_one_if(xy && first), dtx, txc);                                                       \
        tyc = fma(br_one_if(!xy && first), dty, tyc);                                                      \
        tzc = fma(br_one_if(!first), dtz, tzc);                                                            \
        const double len = fmin(t1, tmax) - tc;                                                            \
        if (!(len > BR_MIN_LEN)) dst = junk;                                                               \
        *dst = fmaf(float(len), yv, CUR);                                                                  \
        if (!(t1 < tmax)) break;                                                                           \
        tc = t1;                                                                                           \
    }
                float ca = acc[min(max(off, 0), BR_LAST)], cb;
                for (;;) {
                    KCT_BR_STEP(ca, cb)
                    KCT_BR_STEP(cb, ca)
                }
#undef KCT_BR_STEP
            }
            __syncthreads(); // this pass's sums are complete before its copies take the next angles
            a += m;
        }
    }
    __syncthreads();

    // Add the copies in order and apply the epilogue (or, with an angle
    // split, store this chunk's raw sums).
    double part = 0.0;
    for (int l = threadIdx.x; l < BR_VOX; l += 256) {
        const int li = l % BR_TX, lj = (l / BR_TX) % BR_TY, lk = l / (BR_TX * BR_TY);
        const int i = i0 + li, j = j0 + lj, k = k0 + lk;
        if (i >= ie || j >= je || k >= ke) continue;
        const int c = lk * BR_KS + lj * BR_TX + li;
        const float a_k = ((sums[0][c] + sums[1][c]) + sums[2][c]) + sums[3][c];
        const int64_t idx = (int64_t(k) * g.ny + j) * g.nx + i;
        if (chunks > 1) {
            ep.split[int64_t(chunk) * g.nx * g.ny * g.nz + idx] = a_k;
            continue;
        }
        double o = c0 * double(a_k);
        if (ep.in1 && c1 != 0.0) o += c1 * double(to_f32(static_cast<const TV *>(ep.in1)[idx]));
        if (ep.in2 && c2 != 0.0) o += c2 * double(ep.in2[idx]);
        if (ep.in3 && c3 != 0.0) o += c3 * double(to_f32(static_cast<const TV *>(ep.in3)[idx]));
        const TV st = from_f32<TV>(float(o));
        vol[idx] = st;
        const double sv = double(to_f32(st));
        part += sv * sv;
    }
    if (chunks == 1 && ep.partials) {
        const double sres = block_sum_256b(part, red);
        if (threadIdx.x == 0) ep.partials[logical] = sres;
    }
}

// Sum of the angle chunks' partial volumes in chunk order, then the epilogue
// of k_backward (out = c0 sum + c1 in1 + c2 in2 + c3 in3, partial sums of
// out^2 per workgroup).
template <typename TV>
__global__ __launch_bounds__(256) void k_bwd_combine(const float *__restrict__ split, int chunks, int64_t n,
                                                     TV *__restrict__ vol, Epilogue ep)
{
    __shared__ double red[4];
    if (ep.scal && ep.scal[S_DONE] != 0.0) return;
    double c0 = ep.c[0], c1 = ep.c[1], c2 = ep.c[2], c3 = ep.c[3];
    if (ep.coef_idx >= 0) {
        c0 = ep.scal[ep.coef_idx];
        c1 = ep.scal[ep.coef_idx + 1];
        c2 = ep.scal[ep.coef_idx + 2];
        c3 = ep.scal[ep.coef_idx + 3];
    }
    double part = 0.0;
    for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < n; idx += int64_t(gridDim.x) * 256) {
        float a = 0.f;
#pragma unroll 4
        for (int c = 0; c < chunks; ++c) a += split[int64_t(c) * n + idx];
        double o = c0 * double(a);
        if (ep.in1 && c1 != 0.0) o += c1 * double(to_f32(static_cast<const TV *>(ep.in1)[idx]));
        if (ep.in2 && c2 != 0.0) o += c2 * double(ep.in2[idx]);
        if (ep.in3 && c3 != 0.0) o += c3 * double(to_f32(static_cast<const TV *>(ep.in3)[idx]));
        const TV st = from_f32<TV>(float(o));
        vol[idx] = st;
        const double sv = double(to_f32(st));
        part += sv * sv;
    }
    if (ep.partials) {
        const double s = block_sum_256b(part, red);
        if (threadIdx.x == 0) ep.partials[blockIdx.x] = s;
    }
}

// One voxel per thread up to 2048 workgroups: the split volumes are small.
int64_t combine_groups(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

struct BwdShape {
    int64_t tiles_x, tiles_y, tiles_z, groups;
};

BwdShape bwd_shape(const Plan &p)
{
    static_assert(BR_TX == BWD_TX && BR_TY == BWD_TY, "both back projectors tile x and y alike");
    const int tz = p.bwd_rays ? BR_TZ : p.bwd_kz;
    BwdShape s;
    s.tiles_x = (p.gp.nx + BWD_TX - 1) / BWD_TX;
    s.tiles_y = (p.gp.ny + BWD_TY - 1) / BWD_TY;
    s.tiles_z = (p.gp.nz + tz - 1) / tz;
    s.groups = s.tiles_x * s.tiles_y * s.tiles_z;
    return s;
}

template <typename TP, typename TV, int KZ, int NCM>
kct_status bwd_launch3(Plan &p, const void *proj, void *vol, const Epilogue &ep, hipStream_t st)
{
    const BwdShape s = bwd_shape(p);
    const int64_t launch = ((s.groups + 7) / 8) * 8;
    const int chunks = std::min(p.bwd_asplit, p.gp.na);
    // A dispatch holds fewer than 2^32 work-items (the runtime does not
    // report a larger grid, it truncates it).
    if (launch * 256 * chunks >= (int64_t(1) << 32)) return fail(KCT_E_GEOMETRY, "back projection grid too large");
    if (chunks > 1) {
        if (!ep.split) return fail(KCT_E_INVALID_ARG, "internal: angle-split back projection without a buffer");
        Epilogue raw = ep; // the combine kernel applies the epilogue
        raw.partials = nullptr;
        const dim3 grid(static_cast<unsigned>(launch), static_cast<unsigned>(chunks), 1u);
        if (p.bwd_acc_lds && KZ > 1)
            hipLaunchKernelGGL((k_backward<TP, TV, KZ, NCM, true>), grid, dim3(256),
                               p.bwd_lds + size_t(KZ) * 256 * sizeof(float), st, static_cast<const TP *>(proj),
                               static_cast<TV *>(vol), p.d_tab, p.d_invv, p.d_dlen, p.gp, int(s.tiles_x), int(s.tiles_y),
                               s.groups, p.bwd_pw, p.bwd_ph, p.bwd_fp_angles, p.d_err, p.bwd_xcd_chunk, raw);
        else
            hipLaunchKernelGGL((k_backward<TP, TV, KZ, NCM, false>), grid, dim3(256), p.bwd_lds, st,
                               static_cast<const TP *>(proj), static_cast<TV *>(vol), p.d_tab, p.d_invv, p.d_dlen, p.gp,
                               int(s.tiles_x), int(s.tiles_y), s.groups, p.bwd_pw, p.bwd_ph, p.bwd_fp_angles,
                               p.d_err, p.bwd_xcd_chunk, raw);
        const kct_status e = check_hip(hipGetLastError(), "back projection launch");
        if (e != KCT_OK) return e;
        const int64_t n = p.n_vox();
        hipLaunchKernelGGL((k_bwd_combine<TV>), dim3(unsigned(combine_groups(n))), dim3(256), 0, st, ep.split,
                           chunks, n, static_cast<TV *>(vol), ep);
        return check_hip(hipGetLastError(), "back projection combine launch");
    }
    if (p.bwd_acc_lds && KZ > 1) {
        hipLaunchKernelGGL((k_backward<TP, TV, KZ, NCM, true>), dim3(unsigned(launch)), dim3(256),
                           p.bwd_lds + size_t(KZ) * 256 * sizeof(float), st, static_cast<const TP *>(proj),
                           static_cast<TV *>(vol), p.d_tab, p.d_invv, p.d_dlen, p.gp, int(s.tiles_x), int(s.tiles_y), s.groups,
                           p.bwd_pw, p.bwd_ph, p.bwd_fp_angles, p.d_err, p.bwd_xcd_chunk, ep);
        return check_hip(hipGetLastError(), "back projection launch");
    }
    hipLaunchKernelGGL((k_backward<TP, TV, KZ, NCM, false>), dim3(unsigned(launch)), dim3(256), p.bwd_lds, st,
                       static_cast<const TP *>(proj), static_cast<TV *>(vol), p.d_tab, p.d_invv, p.d_dlen, p.gp,
                       int(s.tiles_x), int(s.tiles_y), s.groups, p.bwd_pw, p.bwd_ph, p.bwd_fp_angles, p.d_err,
                       p.bwd_xcd_chunk, ep);
    return check_hip(hipGetLastError(), "back projection launch");
}

template <typename TP, typename TV, int KZ>
kct_status bwd_launch2(Plan &p, const void *proj, void *vol, const Epilogue &ep, hipStream_t st)
{
    switch (p.bwd_ncmax) {
    case 2: return bwd_launch3<TP, TV, KZ, 2>(p, proj, vol, ep, st);
    case 3: return bwd_launch3<TP, TV, KZ, 3>(p, proj, vol, ep, st);
    case 4: return bwd_launch3<TP, TV, KZ, 4>(p, proj, vol, ep, st);
    case 8: return bwd_launch3<TP, TV, KZ, 8>(p, proj, vol, ep, st);
    case 16: return bwd_launch3<TP, TV, KZ, 16>(p, proj, vol, ep, st);
    }
    return fail(KCT_E_GEOMETRY, "unsupported back projector footprint width");
}

template <typename TP, typename TV>
kct_status bwd_rays_launch(Plan &p, const void *proj, void *vol, const Epilogue &ep, hipStream_t st)
{
    const BwdShape s = bwd_shape(p);
    const int64_t xcd = p.bwd_xcd_chunk;
    const int64_t launch = ((s.groups + 7) / 8) * 8;
    const int chunks = std::min(p.bwd_asplit, p.gp.na);
    if (launch * 256 * chunks >= (int64_t(1) << 32)) return fail(KCT_E_GEOMETRY, "back projection grid too large");
    if (chunks > 1) {
        if (!ep.split) return fail(KCT_E_INVALID_ARG, "internal: angle-split back projection without a buffer");
        Epilogue raw = ep; // the combine kernel applies the epilogue
        raw.partials = nullptr;
        hipLaunchKernelGGL((k_backward_rays<TP, TV>), dim3(unsigned(launch), unsigned(chunks), 1u), dim3(256), 0, st,
                           static_cast<const TP *>(proj), static_cast<TV *>(vol), p.d_tab, p.d_invv, p.d_dlen, p.gp,
                           int(s.tiles_x), int(s.tiles_y), s.groups, xcd, raw);
        const kct_status e = check_hip(hipGetLastError(), "back projection launch");
        if (e != KCT_OK) return e;
        const int64_t n = p.n_vox();
        hipLaunchKernelGGL((k_bwd_combine<TV>), dim3(unsigned(combine_groups(n))), dim3(256), 0, st, ep.split,
                           chunks, n, static_cast<TV *>(vol), ep);
        return check_hip(hipGetLastError(), "back projection combine launch");
    }
    hipLaunchKernelGGL((k_backward_rays<TP, TV>), dim3(unsigned(launch)), dim3(256), 0, st,
                       static_cast<const TP *>(proj), static_cast<TV *>(vol), p.d_tab, p.d_invv, p.d_dlen, p.gp,
                       int(s.tiles_x), int(s.tiles_y), s.groups, xcd, ep);
    return check_hip(hipGetLastError(), "back projection launch");
}

template <typename TP, typename TV>
kct_status bwd_launch1(Plan &p, const void *proj, void *vol, const Epilogue &ep, hipStream_t st)
{
    if (p.bwd_rays) return bwd_rays_launch<TP, TV>(p, proj, vol, ep, st);
    if (p.bwd_kz == 16) return bwd_launch2<TP, TV, 16>(p, proj, vol, ep, st);
    if (p.bwd_kz == 8) return bwd_launch2<TP, TV, 8>(p, proj, vol, ep, st);
    return bwd_launch2<TP, TV, 1>(p, proj, vol, ep, st);
}

// Small volumes make too few tiles to fill 256 CUs (32^3: 128 workgroups);
// their angles are then split over up to 16 chunks of workgroups whose
// partial volumes a second kernel sums in chunk order.  KCT_BWD_SPLIT
// (1..16) overrides the count.
void choose_bwd_split(Plan &p)
{
    const GeoParams &g = p.gp;
    const int64_t groups = bwd_shape(p).groups;
    p.bwd_asplit = 1;
    if (groups < 1024 && g.na > 1)
        p.bwd_asplit = int(std::min<int64_t>({int64_t(16), int64_t(g.na), (2048 + groups - 1) / groups}));
    if (const char *e = std::getenv("KCT_BWD_SPLIT")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 16) p.bwd_asplit = std::min(v, g.na);
    }
}

} // namespace

int64_t bwd_num_groups(const Plan &p)
{
    return std::min(p.bwd_asplit, p.gp.na) > 1 ? combine_groups(p.n_vox()) : bwd_shape(p).groups;
}

int64_t bwd_split_floats(const Plan &p)
{
    const int chunks = std::min(p.bwd_asplit, p.gp.na);
    return chunks > 1 ? int64_t(chunks) * p.n_vox() : 0;
}

// Bounds that size the launch: the widest per-voxel footprint (columns) and
// the largest per-tile detector patch, from the extreme magnification of the
// volume's bounding cylinder.  The kernel clamps to these sizes (and raises a
// flag) if they were ever exceeded, so LDS is never overrun.
kct_status choose_bwd_shape(Plan &p)
{
    const GeoParams &g = p.gp;
    const double xs[2] = {g.X0, g.X0 + g.nx * g.vx}, ys[2] = {g.Y0, g.Y0 + g.ny * g.vy};
    double R = 0.0;
    for (double x : xs)
        for (double y : ys) R = std::max(R, std::sqrt(x * x + y * y));
    const double zmax = std::max(std::fabs(g.Z0), std::fabs(g.Z0 + g.nz * g.vz));
    const double wmin = g.dso - R;
    if (wmin <= 0.0) return fail(KCT_E_GEOMETRY, "volume reaches the source orbit");
    const double mag = g.dsd / wmin * (1.0 + R / wmin);
    const double vox_diag = std::sqrt(g.vx * g.vx + g.vy * g.vy);
    const double ncols = std::floor(vox_diag * mag / g.du + 0.02) + 1.0;
    int ncm = 0;
    for (int c : {2, 3, 4, 8, 16})
        if (ncols <= c) { ncm = c; break; }
    if (!ncm) return fail(KCT_E_GEOMETRY, "voxels project onto more than 16 detector columns");
    p.bwd_ncmax = ncm;

    // Sparse rays: every voxel's footprint narrower than one pixel along u
    // (the column bound above, before its rounding up) and along v (the
    // voxel's height at the nearest depth plus the slope of its farthest
    // plane across its depth), with 2 % to spare.  Then no two rays of one
    // angle meet a voxel, which the ray-driven kernel relies on.
    const double u_width = vox_diag * mag / g.du;
    const double v_height = g.dsd / wmin * (g.vz + zmax * vox_diag / wmin) / g.dv;
    p.bwd_sparse_ok = u_width <= 0.98 && v_height <= 0.98;
    p.bwd_rays = p.bwd_sparse_ok;
    // Tuning override: KCT_BWD_RAYS=0 selects the voxel-driven kernel; 1 the
    // ray-driven one, only where the geometry allows it.
    if (const char *e = std::getenv("KCT_BWD_RAYS")) p.bwd_rays = std::atoi(e) != 0 && p.bwd_sparse_ok;
    // Work order: the XCDs take the tiles in turns of whole rows (at least 32
    // tiles), so that all 8 work on neighbouring rows of one z-layer, whose
    // projection footprints overlap in the MALL, instead of each working
    // through one contiguous eighth of the volume.  1500^3 (ray-driven):
    // 3.25-3.26 against 3.38-3.42 s; 512^3 / 720 angles: 211 against 272 ms
    // (two rows per turn: 215 ms); 256^3 / 360 angles: 14.8 against 15.6 ms
    // (one row of 16 tiles: 15.0 ms).  Tuning override: KCT_BWD_XCD_CHUNK,
    // tiles per turn (-1: one eighth per XCD).
    {
        const int64_t row = (g.nx + BWD_TX - 1) / BWD_TX;
        p.bwd_xcd_chunk = row * ((32 + row - 1) / row);
    }
    if (const char *e = std::getenv("KCT_BWD_XCD_CHUNK")) p.bwd_xcd_chunk = std::max(-1LL, std::atoll(e));

    // The deepest z run per thread (16, else 8 voxels) that still leaves
    // enough workgroups to fill 256 CUs several times over, with the per-voxel
    // sums in LDS (measured fastest on 256^3: 16.0 ms against 17.5 ms for 8
    // voxels, and 20.1 ms for 8 voxels summed in registers, which costs
    // occupancy); one voxel per thread for small volumes.
    const int64_t txy = int64_t((g.nx + BWD_TX - 1) / BWD_TX) * ((g.ny + BWD_TY - 1) / BWD_TY);
    p.bwd_kz = 1;
    for (int kz : {16, 8})
        if (txy * ((g.nz + kz - 1) / kz) >= 2048) {
            p.bwd_kz = kz;
            break;
        }
    p.bwd_acc_lds = true;
    // Tuning overrides: voxels per thread along z (1, 8 or 16) and where the
    // per-voxel sums live (KCT_BWD_ACC=1: LDS, 0: registers).
    if (const char *e = std::getenv("KCT_BWD_KZ")) {
        const int kz = std::atoi(e);
        if (kz == 1 || kz == 8 || kz == 16) p.bwd_kz = kz;
    }
    if (const char *e = std::getenv("KCT_BWD_ACC")) p.bwd_acc_lds = std::atoi(e) != 0;
    // Per-angle tile footprints are kept in LDS for up to 2048 angles.
    p.bwd_fp_angles = std::min(g.na, 2048);
    for (;;) {
        const double tdiag = std::sqrt(std::pow(BWD_TX * g.vx, 2) + std::pow(BWD_TY * g.vy, 2));
        const double pw = std::floor(tdiag * mag / g.du + 0.02) + 2.0;
        const double ph = std::floor(g.dsd * (p.bwd_kz * g.vz / wmin + zmax * tdiag / (wmin * wmin)) / g.dv +
                                     0.02) + 2.0;
        p.bwd_pw = int(std::min<double>(pw, g.nu));
        p.bwd_ph = int(std::min<double>(ph, g.nv));
        // Test hook: a smaller patch-width bound, to exercise the overflow
        // report (every access still stays inside the smaller patch).
        if (const char *e = std::getenv("KCT_BWD_TEST_PW_MAX")) {
            const int v = std::atoi(e);
            if (v >= 1) p.bwd_pw = std::min(p.bwd_pw, v);
        }
        // The patch is followed by NCM zeros that the unrolled column loop
        // may read past its last row.
        p.bwd_lds = size_t(p.bwd_pw) * 16 + size_t(p.bwd_ph) * 8 + size_t(p.bwd_fp_angles) * 16 +
                    (size_t(p.bwd_pw) * p.bwd_ph + size_t(p.bwd_ncmax)) * sizeof(float);
        if (p.bwd_lds + size_t(p.bwd_kz) * 256 * sizeof(float) <= 64 * 1024) {
            choose_bwd_split(p);
            return KCT_OK;
        }
        if (p.bwd_fp_angles > 0) {
            p.bwd_fp_angles = 0;
            continue;
        }
        if (p.bwd_kz == 1) return fail(KCT_E_GEOMETRY, "detector footprint of a voxel tile exceeds LDS");
        p.bwd_kz = p.bwd_kz == 16 ? 8 : 1;
    }
}

kct_status launch_ray_lengths(Plan &p, hipStream_t st)
{
    const int64_t n = int64_t(p.gp.nu) * p.gp.nv;
    const unsigned groups = unsigned(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)));
    hipLaunchKernelGGL(k_ray_lengths, dim3(groups), dim3(256), 0, st, p.d_dlen, p.gp);
    return check_hip(hipGetLastError(), "ray length table launch");
}

kct_status launch_backward(Plan &p, const void *proj, int proj_dtype, void *vol, int vol_dtype,
                           const Epilogue &ep, hipStream_t st)
{
    if (proj_dtype == KCT_F32 && vol_dtype == KCT_F32) return bwd_launch1<float, float>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_BF16 && vol_dtype == KCT_BF16) return bwd_launch1<bf16, bf16>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F16 && vol_dtype == KCT_F16) return bwd_launch1<_Float16, _Float16>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_BF16 && vol_dtype == KCT_F32) return bwd_launch1<bf16, float>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F16 && vol_dtype == KCT_F32) return bwd_launch1<_Float16, float>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F32 && vol_dtype == KCT_BF16) return bwd_launch1<float, bf16>(p, proj, vol, ep, st);
    if (proj_dtype == KCT_F32 && vol_dtype == KCT_F16) return bwd_launch1<float, _Float16>(p, proj, vol, ep, st);
    return fail(KCT_E_DTYPE, "unsupported (projection, volume) storage pair for back projection");
}

} // namespace kct
