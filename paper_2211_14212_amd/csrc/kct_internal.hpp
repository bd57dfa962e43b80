// Internal declarations of the kct library (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kct.h"

namespace kct {

// ---------------------------------------------------------------------------
// Storage types.  All arithmetic happens in float (values) or double
// (geometry, Krylov scalars); these helpers only load and store.
// ---------------------------------------------------------------------------
struct bf16 {
    uint16_t bits;
};

__host__ __device__ inline float to_f32(float v) { return v; }
__host__ __device__ inline float to_f32(bf16 v) {
    uint32_t u = uint32_t(v.bits) << 16;
    return __builtin_bit_cast(float, u);
}
__device__ inline float to_f32(_Float16 v) { return float(v); }

template <typename T> __device__ inline T from_f32(float v);
template <> __device__ inline float from_f32<float>(float v) { return v; }
template <> __device__ inline bf16 from_f32<bf16>(float v) {
    // Round to nearest even on the upper 16 bits; NaN stays a quiet NaN.
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return bf16{uint16_t((u >> 16) | 0x40u)};
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16{uint16_t(u >> 16)};
}
template <> __device__ inline _Float16 from_f32<_Float16>(float v) { return _Float16(v); }

// ---------------------------------------------------------------------------
// Geometry.  Everything the kernels need per gantry angle, computed on the
// host in FP64 (cos/sin evaluated once by the C library).
//   mm frame:    origin on the rotation axis; source (sx, sy, 0).
//   voxel frame: origin at the volume's lower corner, unit = one voxel per
//                axis, so voxel (i,j,k) is [i,i+1) x [j,j+1) x [k,k+1).
// ---------------------------------------------------------------------------
struct alignas(16) AngleGeo {
    double cs, sn;      // cos t, sin t
    double sx, sy;      // source, mm frame
    double svx, svy, svz; // source, voxel frame
    double d0x, d0y;    // (detector centre - source), voxel frame (z component 0)
    double eux, euy;    // e_u per mm of u, voxel frame
    int32_t transposed; // forward projector reads the y-fastest volume copy
    int32_t pad;
};

struct GeoParams {
    int32_t nx, ny, nz, nu, nv, na;
    double vx, vy, vz, du, dv;
    double X0, Y0, Z0;       // lower volume corner, mm frame
    double cu, cv;           // (nu-1)/2, (nv-1)/2
    double dso, dsd;
    double ivz;              // 1/vz
};

// Padded volume copies read by the forward projector: a one-voxel zero
// border on every side, in x-fastest ("normal") and y-fastest
// ("transposed") order.  Element strides of the padded boxes.
struct PadLayout {
    int64_t px, py, pz;   // padded extents nx+2, ny+2, nz+2
    int64_t vox;          // px*py*pz elements per copy
};

// Krylov scalars kept in device FP64 memory.  Fields are addressed by index so
// that kernels of every solver share one layout.
enum ScalarIdx : int {
    S_ALPHA = 0, S_BETA, S_GAMMA, S_DELTA,
    S_RHOBAR, S_PHIBAR, S_PSISQ,
    S_ALPHABAR, S_ZETABAR, S_RHO_OLD, S_RHOBAR_OLD, S_CBAR, S_SBAR,
    S_LAMBDA, S_PNORM2, S_LAST,
    S_DONE, S_ITER, S_HROW, S_KGK, S_RES,
    S_HLAM,                        // lambda reported in history column 4
    S_PREV_EXPL,                   // last explicit residual (stop rule; < 0 before the first)
    S_ERR,                         // 1 once a back projection of this run met a footprint
                                   // wider than the plan's bound (history code 4)
    // Coefficients the scalar kernels leave for the next vector kernels:
    S_F0 = 24, S_F1,               // forward projector epilogue (2)
    S_B0, S_B1, S_B2, S_B3,        // back projector epilogue (4)
    S_V0, S_V1, S_V2, S_V3,        // volume-space update (4)
    S_P0, S_P1,                    // projection-space update (2)
    S_COUNT = 48
};

struct Plan {
    int device = 0;
    kct_geometry geom{};
    std::vector<double> angles;
    std::vector<AngleGeo> host_tab;
    GeoParams gp{};
    PadLayout pad{};
    AngleGeo *d_tab = nullptr;   // per-angle table
    double *d_invv = nullptr;    // 1/v per detector row (0 where v == 0)
    float *d_dlen = nullptr;     // |pixel centre - source| (mm) per detector pixel, [nv][nu]
    void *d_pad = nullptr;       // padded volume copies for plain kct_forward calls (kct_plan_reserve)
    size_t pad_bytes = 0;        // capacity of d_pad
    int *d_err = nullptr;         // back projector footprint overflow flag (0 = fine)
    // Back projector launch shape (chosen from the geometry at plan creation).
    int bwd_kz = 8, bwd_ncmax = 5, bwd_pw = 0, bwd_ph = 0, bwd_fp_angles = 0;
    int bwd_asplit = 1;           // angle chunks of the back projector (small volumes: > 1)
    float *d_split = nullptr;     // partial volumes for plain kct_backproject calls (at plan creation)
    size_t split_bytes = 0;       // capacity of d_split
    int fwd_prefetch = 1;         // forward projector gathers 0, 1 or 2 segments ahead
    int fwd_lane_u = 16;          // forward wave patch: lane_u x (64 / lane_u) rays (64, 32 or 16)
    int fwd_wave_angles = 4;      // angles per forward workgroup: 1 (64 x 4 pixels) or 4, 8, 16 (one patch each)
    int fwd_angle_block = 8;      // forward work order: angles per block (4, 8, 16 or 32)
    int64_t fwd_xcd_chunk = -1;   // forward: logical tiles per XCD turn: -1 one eighth each, 0 half a row band
    bool fwd_pad_f32 = true;      // forward: 16-bit volumes are padded into FP32 copies (small volumes)
    bool bwd_acc_lds = true;      // back projector keeps per-voxel sums in LDS
    bool bwd_sparse_ok = false;   // every voxel footprint narrower than a pixel (u and v)
    bool bwd_rays = false;        // ray-driven back projector (needs bwd_sparse_ok)
    int64_t bwd_xcd_chunk = -1;   // back projector: tiles per XCD turn (-1: one eighth per XCD)
    size_t bwd_lds = 0;
    int64_t n_vox() const { return int64_t(gp.nx) * gp.ny * gp.nz; }
    int64_t n_ray() const { return int64_t(gp.na) * gp.nv * gp.nu; }
};

// Projector epilogue: out = c0*acc + c1*in1 + c2*in2 (+ c3*in3 for the back
// projector), coefficients read from the device scalar block at launch
// (coef_idx >= 0) or taken as given (coef_idx < 0).  Optional FP64 partial
// sum of out^2 per workgroup.
struct Epilogue {
    const double *scal = nullptr; // device scalar block (coefficients, done flag)
    int coef_idx = -1;            // first coefficient index in scal, or -1
    double c[4] = {1.0, 0.0, 0.0, 0.0};
    const void *in1 = nullptr;    // same storage type as out
    const float *in2 = nullptr;   // FP32 (e.g. x)
    const void *in3 = nullptr;    // same storage type as out
    double *partials = nullptr;   // per-workgroup sum of out^2, or null
    float *split = nullptr;       // back projector: bwd_split_floats(plan) floats of partial volumes
    double *err_scal = nullptr;   // back projector: scalar block whose S_ERR records a footprint overflow
};

// Done code a history row records: 4 when a back projection of the run met a
// footprint wider than the plan's bound, else the solver's own S_DONE code.
__device__ inline double hist_code(const double *S) { return S[S_ERR] != 0.0 ? 4.0 : S[S_DONE]; }

// Thread-local error text.
void set_error(const std::string &msg);
kct_status fail(kct_status s, const std::string &msg);
kct_status check_hip(hipError_t e, const char *what);

// Launchers (one per kernel family).  Return KCT_OK or KCT_E_DEVICE.
kct_status launch_pad_volume(Plan &p, const void *vol, int dtype, void *pad, hipStream_t st);
kct_status launch_pad_volume_as(Plan &p, const void *vol, int in_dtype, int out_dtype, void *pad, hipStream_t st);
// Storage of the forward's padded copies for a volume stored in `vol_dtype`:
// FP32 when the plan widens 16-bit volumes (exact, and the FP32 gather is
// faster), else the volume's own type.
inline int fwd_pad_dtype(const Plan &p, int vol_dtype) { return p.fwd_pad_f32 ? int(KCT_F32) : vol_dtype; }
int64_t fwd_num_groups(const Plan &p);
kct_status launch_forward(Plan &p, const void *pad, int vol_dtype, void *proj, int proj_dtype,
                          const Epilogue &ep, hipStream_t st);
int64_t bwd_num_groups(const Plan &p);
// Floats of partial volumes the back projector needs in Epilogue::split (0
// when it does not split the angles).
int64_t bwd_split_floats(const Plan &p);
kct_status launch_backward(Plan &p, const void *proj, int proj_dtype, void *vol, int vol_dtype,
                           const Epilogue &ep, hipStream_t st);
kct_status choose_bwd_shape(Plan &p);
// Fill p.d_dlen (nv * nu floats) on stream `st`.
kct_status launch_ray_lengths(Plan &p, hipStream_t st);

size_t dtype_size(int dt);
bool dtype_ok(int dt);

} // namespace kct

// Plans with at least this many angles take the forward work order of
// 128-angle blocks handed to the XCDs in half row bands.
constexpr int FWD_ORDER_MIN_ANGLES = 256;

// The opaque handle of kct.h is the plan itself.
struct kct_plan : public kct::Plan {};
