// Forward cone-beam projection y = A x (Siddon path lengths), gfx950.
//
// One thread traces one ray (source -> pixel centre) through the voxel grid
// and accumulates length * value in FP32.  The ray geometry (entry point,
// plane crossings) is evaluated in FP64, which runs at the non-packed FP32
// rate on CDNA4, so the per-coefficient length carries ~1e-16 relative error
// instead of the ~1e-5 an FP32 parametrisation of a 256-voxel ray would.
//
// Launch shape: each wave traces a compact patch of neighbouring pixels of
// one angle (16 x 4 by default), so its lanes follow rays that cross the same
// voxel columns.  By default a workgroup's 4 waves trace the same patch at 4
// consecutive angles (wave_angles = 4; 8 in workgroups of 512 threads for
// large volumes): rays of neighbouring angles through one pixel nearly
// coincide, so those waves gather the same lines at nearly the same time and
// the CU's L1 and the XCD's L2 serve them once.  (The
// alternative, 4 waves tiling a 64 x 4 pixel block of one angle, is 20 %
// slower on 256^3 / 360 x 512^2 and 60 % slower on a 1500^3 volume whose
// gathers then miss L2 half of the time.)  Lanes map to u, and neighbouring u
// are displaced along e_u, which is close to y for angles with |cos| >= |sin|:
// for those angles the kernel reads a y-fastest copy of the volume so that a
// wave's gather touches a few contiguous runs instead of 64 scattered lines.
// Both copies carry a one-voxel zero border, which makes a one-step overshoot
// at the exit face (possible when a crossing rounds to just before the exit
// parameter) read zero instead of leaving the buffer.
//
// Workgroups are renumbered so that the 8 XCDs (round-robin dispatch) each
// take a contiguous range of the work order below, in which neighbouring
// workgroups trace neighbouring angles and detector rows (see k_forward).

#include "kct_internal.hpp"

#include <algorithm>

namespace kct {

namespace {

constexpr int FWD_TU = 64; // detector columns per workgroup
constexpr int FWD_TV = 4;  // detector rows per workgroup

// --------------------------------------------------------------------------
// Padded volume copies: out[0:vox] x-fastest, out[vox:2vox] y-fastest, both
// (nz+2) x (ny+2) x (nx+2) with a zero border.  32x32 xy tiles through LDS
// so that both writes are coalesced.
// --------------------------------------------------------------------------
template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void k_pad_volume(const TIN *__restrict__ in, TOUT *__restrict__ out,
                                                    int nx, int ny, int nz, PadLayout pl)
{
    __shared__ float tile[32][33];
    const int tiles_x = int((pl.px + 31) / 32);
    const int bx = blockIdx.x % tiles_x, by = blockIdx.x / tiles_x;
    const int64_t pk = blockIdx.y; // padded z index
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5; // 32 x 8
    const int64_t k = pk - 1;
    // Load: padded (pi, pj) = (bx*32 + tx, by*32 + ty + 8r).
    for (int r = 0; r < 4; ++r) {
        const int64_t pi = int64_t(bx) * 32 + tx, pj = int64_t(by) * 32 + ty + 8 * r;
        float v = 0.f;
        const int64_t i = pi - 1, j = pj - 1;
        if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz)
            v = to_f32(in[(k * ny + j) * nx + i]);
        tile[ty + 8 * r][tx] = v;
        if (pi < pl.px && pj < pl.py) out[(pk * pl.py + pj) * pl.px + pi] = from_f32<TOUT>(v);
    }
    __syncthreads();
    // Transposed write: element (pk, pi, pj) at (pk*px + pi)*py + pj, pj fastest.
    for (int r = 0; r < 4; ++r) {
        const int64_t pj = int64_t(by) * 32 + tx, pi = int64_t(bx) * 32 + ty + 8 * r;
        if (pi < pl.px && pj < pl.py)
            out[pl.vox + (pk * pl.px + pi) * pl.py + pj] = from_f32<TOUT>(tile[tx][ty + 8 * r]);
    }
}

// Deterministic workgroup sum of one double per thread (256, 512 or 1024
// threads; `red` holds one double per wave): waves summed in groups of four,
// the groups in order.
__device__ inline double block_sum(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = int(blockDim.x) >> 6;
        for (int q = 0; q < nw; q += 4) s += ((red[q] + red[q + 1]) + red[q + 2]) + red[q + 3];
    }
    return s;
}

constexpr int64_t FWD_MAX_BLOCKS = int64_t(1) << 20; // 2^28 work-items per dispatch

// 0.0 or 1.0 from a predicate, built from the high word only (one select).
__device__ inline double one_if(bool c)
{
    return __builtin_bit_cast(double, uint64_t(c ? 0x3ff00000u : 0u) << 32);
}

// Work order: blocks of angle_block angles (8 by default); inside a block,
// detector row bands (4 rows, or one wave patch's rows with wave_angles = 4);
// inside a band, the block's angles (in groups of 4 with wave_angles = 4) and
// the u tiles.  With one angle per workgroup the angles are the slower index,
// with 4 the u tiles are, so that the workgroups holding the block's angles
// of one patch start together.  The ~256 workgroups an XCD keeps in flight
// then cover a few row bands of a handful of neighbouring angles, whose rays
// cross the same few z-slices of the volume.

// One workgroup tile (logical workgroup index `logical`): 64 x 4 pixels of
// one angle, or a lane_u x (64 / lane_u) patch at 4 angles.
template <typename TV, typename TP, typename OFF, int DEPTH>
__device__ inline void fwd_tile(const TV *__restrict__ vpad, TP *__restrict__ proj, const AngleGeo *__restrict__ tab,
                                const GeoParams &g, const PadLayout &pl, int tiles_u, int tiles_v, int lane_u,
                                int wave_angles, int angle_block, int64_t logical,
                                const Epilogue &ep, double *red)
{
    double c0 = ep.c[0], c1 = ep.c[1];
    if (ep.coef_idx >= 0) {
        c0 = ep.scal[ep.coef_idx];
        c1 = ep.scal[ep.coef_idx + 1];
    }

    // Each wave traces a lane_u x (64 / lane_u) patch (16 x 4 by default).
    // Rays of adjacent rows follow nearly the same voxels, so a compact patch
    // sends fewer requests per gather to L2 than a 64-wide row does: on
    // 256^3 / 360 x 512^2, 5.4 instead of 6.5 L2 requests per gather and 20.6
    // instead of 22.7 ms per projection.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int rows_w = 64 / lane_u;
    const int n_at = angle_block / wave_angles; // angle groups per block
    const int per_band = n_at * tiles_u;
    const int per_block = per_band * tiles_v;
    const int ab = int(logical / per_block);
    const int r1 = int(logical - int64_t(ab) * per_block);
    const int tvi = r1 / per_band;
    const int r2 = r1 - tvi * per_band;
    int a, iu, iv;
    if (wave_angles == 1) { // tiles of 64 x 4 pixels; waves tile them
        const int ai = r2 / tiles_u, tui = r2 - ai * tiles_u;
        const int waves_u = FWD_TU / lane_u;
        a = ab * angle_block + ai;
        iu = tui * FWD_TU + (wv % waves_u) * lane_u + lane % lane_u;
        iv = tvi * FWD_TV + (wv / waves_u) * rows_w + lane / lane_u;
    } else { // tiles of one wave patch; wave w takes angle wave_angles * group + w
        const int tui = r2 / n_at, ag = r2 - tui * n_at;
        a = ab * angle_block + ag * wave_angles + wv;
        iu = tui * lane_u + lane % lane_u;
        iv = tvi * rows_w + lane / lane_u;
    }
    // The angle is uniform over the wave; saying so keeps its table row in
    // scalar registers.
    a = __builtin_amdgcn_readfirstlane(a);
    const bool valid = a < g.na && iu < g.nu && iv < g.nv;

    float acc = 0.f;
    double dn = 0.0;
    if (valid) {
        const AngleGeo A = tab[a];
        const double u = (iu - g.cu) * g.du, v = (iv - g.cv) * g.dv;
        const double dx = A.d0x + u * A.eux, dy = A.d0y + u * A.euy, dz = v * g.ivz;
        dn = sqrt(g.dsd * g.dsd + u * u + v * v);
        double tmin = 0.0, tmax = 1.0;
        double inx = 0.0, iny = 0.0, inz = 0.0;
        if (dx != 0.0) {
            inx = 1.0 / dx;
            const double t0 = (0.0 - A.svx) * inx, t1 = (double(g.nx) - A.svx) * inx;
            tmin = fmax(tmin, fmin(t0, t1));
            tmax = fmin(tmax, fmax(t0, t1));
        } else if (!(A.svx >= 0.0 && A.svx < g.nx)) {
            tmax = -1.0;
        }
        if (dy != 0.0) {
            iny = 1.0 / dy;
            const double t0 = (0.0 - A.svy) * iny, t1 = (double(g.ny) - A.svy) * iny;
            tmin = fmax(tmin, fmin(t0, t1));
            tmax = fmin(tmax, fmax(t0, t1));
        } else if (!(A.svy >= 0.0 && A.svy < g.ny)) {
            tmax = -1.0;
        }
        if (dz != 0.0) {
            inz = 1.0 / dz;
            const double t0 = (0.0 - A.svz) * inz, t1 = (double(g.nz) - A.svz) * inz;
            tmin = fmax(tmin, fmin(t0, t1));
            tmax = fmin(tmax, fmax(t0, t1));
        } else if (!(A.svz >= 0.0 && A.svz < g.nz)) {
            tmax = -1.0;
        }
        if (tmin < tmax) {
            const int i = min(max(int(floor(A.svx + tmin * dx)), 0), g.nx - 1);
            const int j = min(max(int(floor(A.svy + tmin * dy)), 0), g.ny - 1);
            const int k = min(max(int(floor(A.svz + tmin * dz)), 0), g.nz - 1);
            // Byte strides of the chosen padded copy.
            constexpr int64_t ES = sizeof(TV);
            const int64_t sx = (A.transposed ? pl.py : 1) * ES;
            const int64_t sy = (A.transposed ? 1 : pl.px) * ES;
            const int64_t sz = pl.px * pl.py * ES;
            const int64_t base = (A.transposed ? pl.vox : 0) * ES;
            constexpr double FAR = 1.0e300;
            double tx = FAR, ty = FAR, tz = FAR, dtx = 0.0, dty = 0.0, dtz = 0.0;
            OFF stx = 0, sty = 0, stz = 0;
            if (dx > 0.0) { tx = (i + 1 - A.svx) * inx; dtx = inx; stx = OFF(sx); }
            else if (dx < 0.0) { tx = (i - A.svx) * inx; dtx = -inx; stx = OFF(-sx); }
            if (dy > 0.0) { ty = (j + 1 - A.svy) * iny; dty = iny; sty = OFF(sy); }
            else if (dy < 0.0) { ty = (j - A.svy) * iny; dty = -iny; sty = OFF(-sy); }
            if (dz > 0.0) { tz = (k + 1 - A.svz) * inz; dtz = inz; stz = OFF(sz); }
            else if (dz < 0.0) { tz = (k - A.svz) * inz; dtz = -inz; stz = OFF(-sz); }
            OFF off = OFF(base + (i + 1) * sx + (j + 1) * sy + (k + 1) * sz);
            const char *vb = reinterpret_cast<const char *>(vpad);
            double tc = tmin;
            // Termination: while tc < tmax, the nearest crossing tn is one of
            // tx, ty, tz (all >= tc) and that axis then advances by its
            // step 1/|d| >= v/|pixel - source| > 0, so tc reaches tmax after at
            // most nx+ny+nz+3 crossings.  Every access stays inside the padded
            // copy: indices start inside the volume and at most one step per
            // axis can land on the zero border before tc reaches tmax.
            if constexpr (DEPTH == 2) {
                // Two gathers in flight.  The walker runs one voxel ahead of
                // the sums: while the segment of voxel n is added, the values
                // of voxels n+1 and n+2 are on their way.  Three registers
                // rotate through an unrolled trip and hold the raw stored
                // values (a conversion right after a load would wait for it),
                // so no register is copied while its load is pending.  The
                // trip has no per-lane exit: a lane that has reached tmax stays
                // in the loop with its sums frozen until every lane of the
                // wave has, so the loop's only branch is wave-uniform and each
                // use waits for its own load only.  The walker steps only
                // while the current voxel's exit lies before tmax (the rule
                // of the loops below, which keeps every index inside the
                // padded copy); otherwise the load repeats the current voxel.
                // Segments are added in the same order with the same
                // operations as the one-ahead loop: the sums are bitwise
                // equal.
                TV r0 = *reinterpret_cast<const TV *>(vb + off), r1 = r0, r2 = r0;
                double ta = tc, tb;
                bool alive;
                {
                    const double m1 = fmin(tx, ty);
                    tb = fmin(m1, tz);
                    alive = tb < tmax;
                    const bool xy = tx <= ty, first = m1 <= tz;
                    tx = fma(one_if(alive && xy && first), dtx, tx);
                    ty = fma(one_if(alive && !xy && first), dty, ty);
                    tz = fma(one_if(alive && !first), dtz, tz);
                    off += alive ? (first ? (xy ? stx : sty) : stz) : OFF(0);
                    r1 = *reinterpret_cast<const TV *>(vb + off);
                    if (!alive) acc = fmaf(float(tmax - ta), to_f32(r0), acc);
                }
#define KCT_FWD2_STEP(R0, R1, R2)                                                                          \
    {                                                                                                      \
        const double m1 = fmin(tx, ty);                                                                    \
        const double tcx = fmin(m1, tz);                                                                   \
        const bool more = alive && tcx < tmax;                                                             \
        const bool xy = tx <= ty, first = m1 <= tz;                                                        \
        tx = fma(one_if(more && xy && first), dtx, tx);                                                    \
        ty = fma(one_if(more && !xy && first), dty, ty);                                                   \
        tz = fma(one_if(more && !first), dtz, tz);                                                         \
        off += more ? (first ? (xy ? stx : sty) : stz) : OFF(0);                                           \
        R2 = *reinterpret_cast<const TV *>(vb + off);                                                      \
        const float s0 = fmaf(float(tb - ta), to_f32(R0), acc);                                            \
        const float s1 = fmaf(float(tmax - tb), to_f32(R1), s0);                                           \
        acc = alive ? (more ? s0 : s1) : acc;                                                              \
        alive = more;                                                                                      \
        ta = tb;                                                                                           \
        tb = tcx;                                                                                          \
    }
                while (__any(alive)) {
                    KCT_FWD2_STEP(r0, r1, r2)
                    KCT_FWD2_STEP(r1, r2, r0)
                    KCT_FWD2_STEP(r2, r0, r1)
                }
#undef KCT_FWD2_STEP
            } else if constexpr (DEPTH == 1) {
                // Two segments per trip, so the voxel value is requested a
                // whole step before its FMA and no register is copied.  Each
                // step advances exactly one axis, the one whose crossing comes
                // first (x before y before z on ties; a tie then yields a
                // zero-length segment in a diagonal neighbour, which adds
                // exactly 0).  A lane whose next crossing lies at or beyond
                // tmax adds its last segment, up to tmax, and leaves the loop.
                float va = to_f32(*reinterpret_cast<const TV *>(vb + off));
                for (;;) {
                    const double m1 = fmin(tx, ty);
                    const double t1 = fmin(m1, tz);
                    if (!(t1 < tmax)) {
                        acc = fmaf(float(tmax - tc), va, acc);
                        break;
                    }
                    {
                        const bool xy = tx <= ty, first = m1 <= tz;
                        tx = fma(one_if(xy && first), dtx, tx);
                        ty = fma(one_if(!xy && first), dty, ty);
                        tz = fma(one_if(!first), dtz, tz);
                        off += first ? (xy ? stx : sty) : stz;
                    }
                    const float vb1 = to_f32(*reinterpret_cast<const TV *>(vb + off));
                    acc = fmaf(float(t1 - tc), va, acc);
                    const double m2 = fmin(tx, ty);
                    const double t2 = fmin(m2, tz);
                    if (!(t2 < tmax)) {
                        acc = fmaf(float(tmax - t1), vb1, acc);
                        break;
                    }
                    {
                        const bool xy = tx <= ty, first = m2 <= tz;
                        tx = fma(one_if(xy && first), dtx, tx);
                        ty = fma(one_if(!xy && first), dty, ty);
                        tz = fma(one_if(!first), dtz, tz);
                        off += first ? (xy ? stx : sty) : stz;
                    }
                    va = to_f32(*reinterpret_cast<const TV *>(vb + off));
                    acc = fmaf(float(t2 - t1), vb1, acc);
                    tc = t2;
                }
            } else {
                for (;;) {
                    const double tn = fmin(fmin(tx, ty), fmin(tz, tmax));
                    const float val = to_f32(*reinterpret_cast<const TV *>(vb + off));
                    acc = fmaf(float(tn - tc), val, acc);
                    tc = tn;
                    if (!(tc < tmax)) break;
                    const bool cx = tx <= tn, cy = ty <= tn, cz = tz <= tn;
                    tx = fma(one_if(cx), dtx, tx);
                    ty = fma(one_if(cy), dty, ty);
                    tz = fma(one_if(cz), dtz, tz);
                    off += (cx ? stx : OFF(0)) + (cy ? sty : OFF(0)) + (cz ? stz : OFF(0));
                }
            }
        }
    }

    float outv = 0.f;
    if (valid) {
        const int64_t ray = (int64_t(a) * g.nv + iv) * g.nu + iu;
        double o = c0 * (double(acc) * dn);
        if (ep.in1 && c1 != 0.0) o += c1 * double(to_f32(static_cast<const TP *>(ep.in1)[ray]));
        const TP st = from_f32<TP>(float(o));
        proj[ray] = st;
        outv = to_f32(st);
    }
    if (ep.partials) {
        const double s = block_sum(double(outv) * double(outv), red);
        if (threadIdx.x == 0) ep.partials[logical] = s;
    }
}

// A dispatch holds fewer than 2^32 work-items, so large problems launch at
// most FWD_MAX_BLOCKS workgroups (a multiple of 8) and each takes the tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...  The physical index b keeps its XCD
// (b mod 8) on every pass.  The XCDs take the logical tiles in turns of
// xcd_chunk consecutive tiles: with xcd_chunk = launch / 8 each XCD works
// through one contiguous eighth (neighbouring angles and detector rows share
// its L2); with half a row band per turn all XCDs work on neighbouring rows
// of the same angle block at once (their rays cross the same few z-slices,
// which stay in the MALL).
// Workgroups of 256 threads, or 64 per angle with 8 or 16 angles each (the
// bound lets the compiler budget registers for up to 1024).
template <typename TV, typename TP, typename OFF, int DEPTH>
__global__ __launch_bounds__(1024) void k_forward(const TV *__restrict__ vpad, TP *__restrict__ proj,
                                                 const AngleGeo *__restrict__ tab, GeoParams g, PadLayout pl,
                                                 int tiles_u, int tiles_v, int lane_u, int wave_angles,
                                                 int angle_block, int64_t groups, int64_t launch,
                                                 int64_t xcd_chunk, Epilogue ep)
{
    __shared__ double red[16];
    if (ep.scal && ep.scal[S_DONE] != 0.0) return;
    const int64_t g8 = launch >> 3;
    const int64_t C = xcd_chunk > 0 ? xcd_chunk : g8;
    for (int64_t b = blockIdx.x; b < launch; b += gridDim.x) {
        // The k-th workgroup of XCD x takes chunk q = k / C: logical tiles
        // q * 8C + x * w + k mod C, w = min(C, g8 - q * C) (a bijection onto
        // [0, launch)).
        const int64_t k = b >> 3, q = k / C, r = k - q * C;
        const int64_t w = min(C, g8 - q * C);
        const int64_t logical = q * 8 * C + (b & 7) * w + r;
        if (logical >= groups) continue;
        fwd_tile<TV, TP, OFF, DEPTH>(vpad, proj, tab, g, pl, tiles_u, tiles_v, lane_u, wave_angles, angle_block,
                                         logical, ep, red);
        __syncthreads(); // red[] is reused by the next tile's reduction
    }
}

// Workgroup tiles along u and v, and the workgroup count: 64 x 4 pixel
// tiles of single angles, or wave-patch tiles of 4 angles.
int64_t fwd_tiling(const Plan &p, int &tiles_u, int &tiles_v)
{
    const int tu = p.fwd_wave_angles == 1 ? FWD_TU : p.fwd_lane_u;
    const int tv = p.fwd_wave_angles == 1 ? FWD_TV : 64 / p.fwd_lane_u;
    tiles_u = (p.gp.nu + tu - 1) / tu;
    tiles_v = (p.gp.nv + tv - 1) / tv;
    const int64_t blocks = (p.gp.na + p.fwd_angle_block - 1) / p.fwd_angle_block;
    return blocks * (p.fwd_angle_block / p.fwd_wave_angles) * tiles_u * tiles_v;
}

template <typename TIN, typename TOUT>
kct_status pad_typed(Plan &p, const void *vol, void *pad, hipStream_t st)
{
    const int tiles_x = int((p.pad.px + 31) / 32), tiles_y = int((p.pad.py + 31) / 32);
    dim3 grid(unsigned(tiles_x * tiles_y), unsigned(p.pad.pz));
    hipLaunchKernelGGL((k_pad_volume<TIN, TOUT>), grid, dim3(256), 0, st, static_cast<const TIN *>(vol),
                       static_cast<TOUT *>(pad), p.gp.nx, p.gp.ny, p.gp.nz, p.pad);
    return check_hip(hipGetLastError(), "pad volume launch");
}

template <typename TV, typename TP>
kct_status fwd_typed(Plan &p, const void *pad, void *proj, const Epilogue &ep, hipStream_t st)
{
    int tiles_u = 0, tiles_v = 0;
    const int64_t groups = fwd_tiling(p, tiles_u, tiles_v);
    const int64_t launch = ((groups + 7) / 8) * 8;
    const int64_t per_band = int64_t(p.fwd_angle_block / p.fwd_wave_angles) * tiles_u;
    const int64_t xcd_chunk = p.fwd_xcd_chunk > 0 ? p.fwd_xcd_chunk
                              : p.fwd_xcd_chunk < 0 ? 0 : std::max<int64_t>(1, per_band / 2);
    const unsigned grid = unsigned(std::min<int64_t>(launch, FWD_MAX_BLOCKS));
    const unsigned threads = unsigned(p.fwd_wave_angles > 4 ? 64 * p.fwd_wave_angles : 256);
    // 32-bit byte offsets when both padded copies fit in 4 GiB.
    const bool small = 2 * p.pad.vox * int64_t(sizeof(TV)) < int64_t(0xffffffffLL);
#define KCT_FWD_LAUNCH(OFF_T, PF)                                                                                  \
    hipLaunchKernelGGL((k_forward<TV, TP, OFF_T, PF>), dim3(grid), dim3(threads), 0, st, static_cast<const TV *>(pad), \
                       static_cast<TP *>(proj), p.d_tab, p.gp, p.pad, tiles_u, tiles_v, p.fwd_lane_u,                 \
                       p.fwd_wave_angles, p.fwd_angle_block, groups, launch, xcd_chunk, ep)
    if (small) {
        if (p.fwd_prefetch == 2) KCT_FWD_LAUNCH(uint32_t, 2);
        else if (p.fwd_prefetch == 1) KCT_FWD_LAUNCH(uint32_t, 1);
        else KCT_FWD_LAUNCH(uint32_t, 0);
    } else {
        if (p.fwd_prefetch == 2) KCT_FWD_LAUNCH(uint64_t, 2);
        else if (p.fwd_prefetch == 1) KCT_FWD_LAUNCH(uint64_t, 1);
        else KCT_FWD_LAUNCH(uint64_t, 0);
    }
#undef KCT_FWD_LAUNCH
    return check_hip(hipGetLastError(), "forward projection launch");
}

template <typename TIN>
kct_status pad_dispatch_out(Plan &p, const void *vol, int out_dt, void *pad, hipStream_t st)
{
    switch (out_dt) {
    case KCT_F32: return pad_typed<TIN, float>(p, vol, pad, st);
    case KCT_BF16: return pad_typed<TIN, bf16>(p, vol, pad, st);
    case KCT_F16: return pad_typed<TIN, _Float16>(p, vol, pad, st);
    }
    return fail(KCT_E_DTYPE, "unsupported volume storage type");
}

template <typename TV>
kct_status fwd_dispatch_proj(Plan &p, const void *pad, void *proj, int proj_dt, const Epilogue &ep,
                             hipStream_t st)
{
    switch (proj_dt) {
    case KCT_F32: return fwd_typed<TV, float>(p, pad, proj, ep, st);
    case KCT_BF16: return fwd_typed<TV, bf16>(p, pad, proj, ep, st);
    case KCT_F16: return fwd_typed<TV, _Float16>(p, pad, proj, ep, st);
    }
    return fail(KCT_E_DTYPE, "unsupported projection storage type");
}

} // namespace

// Build both padded copies of `vol` (storage `dtype`) in `pad`, stored in
// the same type.  `pad` must hold 2 * pad.vox elements of that type.
kct_status launch_pad_volume(Plan &p, const void *vol, int dtype, void *pad, hipStream_t st)
{
    switch (dtype) {
    case KCT_F32: return pad_dispatch_out<float>(p, vol, dtype, pad, st);
    case KCT_BF16: return pad_dispatch_out<bf16>(p, vol, dtype, pad, st);
    case KCT_F16: return pad_dispatch_out<_Float16>(p, vol, dtype, pad, st);
    }
    return fail(KCT_E_DTYPE, "unsupported volume storage type");
}

// As launch_pad_volume, converting from `in_dtype` to `out_dtype` storage.
kct_status launch_pad_volume_as(Plan &p, const void *vol, int in_dtype, int out_dtype, void *pad, hipStream_t st)
{
    switch (in_dtype) {
    case KCT_F32: return pad_dispatch_out<float>(p, vol, out_dtype, pad, st);
    case KCT_BF16: return pad_dispatch_out<bf16>(p, vol, out_dtype, pad, st);
    case KCT_F16: return pad_dispatch_out<_Float16>(p, vol, out_dtype, pad, st);
    }
    return fail(KCT_E_DTYPE, "unsupported volume storage type");
}

int64_t fwd_num_groups(const Plan &p)
{
    int tiles_u = 0, tiles_v = 0;
    return fwd_tiling(p, tiles_u, tiles_v);
}

// Project the padded copies in `pad` (built by launch_pad_volume with
// `vol_dtype`) into `proj`, applying the epilogue.
kct_status launch_forward(Plan &p, const void *pad, int vol_dtype, void *proj, int proj_dtype,
                          const Epilogue &ep, hipStream_t st)
{
    switch (vol_dtype) {
    case KCT_F32: return fwd_dispatch_proj<float>(p, pad, proj, proj_dtype, ep, st);
    case KCT_BF16: return fwd_dispatch_proj<bf16>(p, pad, proj, proj_dtype, ep, st);
    case KCT_F16: return fwd_dispatch_proj<_Float16>(p, pad, proj, proj_dtype, ep, st);
    }
    return fail(KCT_E_DTYPE, "unsupported volume storage type");
}

} // namespace kct
