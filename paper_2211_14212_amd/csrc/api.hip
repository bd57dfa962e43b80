// Plan creation, geometry validation, errors and the plain projector calls.

#include "gmres.hpp"
#include "kct_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

namespace kct {

namespace {
thread_local std::string g_last_error;

// Makes the plan's device current for the duration of a call and restores
// the caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Scratch of kct_forward_noalloc: the forward projector's padded volume
// copies in a device array the library owns (each GPU the library runs on
// holds its own copy of it until the process ends).  In host code the array's
// name is not a device address: the address of each GPU's copy is resolved
// once per device, at plan creation with that device current, and kept in
// g_scratch; only those addresses are passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = KCT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[SCRATCH_DEVICES] = {};
bool g_scratch_tried[SCRATCH_DEVICES] = {};

// With device `dev` current.  A failure leaves the address unset, which
// kct_forward_noalloc then reports; the plan itself does not depend on it.
void resolve_scratch(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= SCRATCH_DEVICES || g_scratch_tried[dev]) return;
    g_scratch_tried[dev] = true;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) g_scratch[dev] = ptr;
    else (void)hipGetLastError(); // do not leave the failure for the caller's next HIP call
}

void *scratch_address(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (dev >= 0 && dev < SCRATCH_DEVICES) ? g_scratch[dev] : nullptr;
}
} // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

kct_status fail(kct_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

kct_status check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return KCT_OK;
    return fail(e == hipErrorOutOfMemory ? KCT_E_OOM : KCT_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

size_t dtype_size(int dt) { return dt == KCT_F32 ? 4 : 2; }
bool dtype_ok(int dt) { return dt == KCT_F32 || dt == KCT_BF16 || dt == KCT_F16; }

static kct_status validate(const kct_geometry *g)
{
    if (!g) return fail(KCT_E_INVALID_ARG, "geometry is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return fail(KCT_E_GEOMETRY, "volume size must be positive");
    if (g->nu <= 0 || g->nv <= 0) return fail(KCT_E_GEOMETRY, "detector size must be positive");
    if (g->n_angles <= 0) return fail(KCT_E_GEOMETRY, "n_angles must be positive");
    if (!g->angles) return fail(KCT_E_INVALID_ARG, "angles is NULL");
    if (!finite_pos(g->vx) || !finite_pos(g->vy) || !finite_pos(g->vz))
        return fail(KCT_E_GEOMETRY, "voxel size must be positive and finite");
    if (!finite_pos(g->du) || !finite_pos(g->dv)) return fail(KCT_E_GEOMETRY, "pixel pitch must be positive");
    if (!std::isfinite(g->ox) || !std::isfinite(g->oy) || !std::isfinite(g->oz))
        return fail(KCT_E_GEOMETRY, "volume offset must be finite");
    if (!finite_pos(g->dso)) return fail(KCT_E_GEOMETRY, "DSO must be positive");
    if (!(std::isfinite(g->dsd) && g->dsd > g->dso)) return fail(KCT_E_GEOMETRY, "DSD must exceed DSO");
    for (int a = 0; a < g->n_angles; ++a)
        if (!std::isfinite(g->angles[a])) return fail(KCT_E_GEOMETRY, "angles must be finite");
    const double X0 = g->ox - 0.5 * g->nx * g->vx, Y0 = g->oy - 0.5 * g->ny * g->vy;
    double R = 0.0;
    for (double x : {X0, X0 + g->nx * g->vx})
        for (double y : {Y0, Y0 + g->ny * g->vy}) R = std::max(R, std::sqrt(x * x + y * y));
    if (R >= g->dso) return fail(KCT_E_GEOMETRY, "the volume reaches the source orbit (need radius < DSO)");
    if (R >= g->dsd - g->dso) return fail(KCT_E_GEOMETRY, "the volume reaches the detector (need radius < DSD-DSO)");
    const double nray = double(g->n_angles) * g->nu * g->nv;
    if (nray > 4.0e12) return fail(KCT_E_GEOMETRY, "too many rays");
    return KCT_OK;
}

static void build_tables(Plan &p)
{
    const kct_geometry &g = p.geom;
    GeoParams &gp = p.gp;
    gp.nx = g.nx; gp.ny = g.ny; gp.nz = g.nz; gp.nu = g.nu; gp.nv = g.nv; gp.na = g.n_angles;
    gp.vx = g.vx; gp.vy = g.vy; gp.vz = g.vz; gp.du = g.du; gp.dv = g.dv;
    gp.X0 = g.ox - 0.5 * g.nx * g.vx;
    gp.Y0 = g.oy - 0.5 * g.ny * g.vy;
    gp.Z0 = g.oz - 0.5 * g.nz * g.vz;
    gp.cu = 0.5 * (g.nu - 1);
    gp.cv = 0.5 * (g.nv - 1);
    gp.dso = g.dso; gp.dsd = g.dsd;
    gp.ivz = 1.0 / g.vz;
    p.host_tab.resize(g.n_angles);
    for (int a = 0; a < g.n_angles; ++a) {
        const double cs = std::cos(p.angles[a]), sn = std::sin(p.angles[a]);
        AngleGeo &A = p.host_tab[a];
        A.cs = cs; A.sn = sn;
        A.sx = g.dso * cs; A.sy = g.dso * sn;
        A.svx = (A.sx - gp.X0) / g.vx;
        A.svy = (A.sy - gp.Y0) / g.vy;
        A.svz = (0.0 - gp.Z0) / g.vz;
        A.d0x = -g.dsd * cs / g.vx;
        A.d0y = -g.dsd * sn / g.vy;
        A.eux = -sn / g.vx;
        A.euy = cs / g.vy;
        // Rays run mostly along x when |cos| >= |sin|; neighbouring pixels are
        // then displaced along y, so the y-fastest copy keeps a wave coalesced.
        A.transposed = std::fabs(cs) >= std::fabs(sn) ? 1 : 0;
        A.pad = 0;
    }
    p.pad.px = g.nx + 2;
    p.pad.py = g.ny + 2;
    p.pad.pz = g.nz + 2;
    p.pad.vox = p.pad.px * p.pad.py * p.pad.pz;
}

// The forward projector's launch shape for the plan's geometry, then the
// tuning overrides from the environment.
void choose_fwd_shape(Plan &p)
{
    const kct_geometry &g = p.geom;
    // Forward wave patch: when neighbouring rays are at least a voxel apart
    // at the rotation axis, a wider, flatter patch (32 x 2 pixels) touches
    // fewer lines per gather than 16 x 4 (1500^3 at 10 um, 0.1 mm pixels at
    // magnification 5.3: 3.65 against 3.93 s); with finer ray spacing 16 x 4
    // is faster (256^3 at 0.5 mm, 0.4 mm pixels at 1.5: 17.3 against 17.8 ms).
    if (g.du * g.dso / g.dsd >= std::min(g.vx, g.vy)) p.fwd_lane_u = 32;
    // 16-bit volumes: FP32 padded copies gather faster while they are small
    // (512^3: 240 against 290 ms per projection); once the FP32 copies pass
    // 4 GiB, the 16-bit copies' halved gather traffic wins (1500^3: 3.64
    // against 3.92 s).
    p.fwd_pad_f32 = 2 * p.pad.vox * int64_t(sizeof(float)) < int64_t(0xffffffffLL);
    // Gathers in flight: two segments ahead where the padded copies stay
    // 16-bit (the volume is large and a fraction of the gathers go to HBM:
    // 1500^3, 3.50 -> 3.33 s), else one (the FP32-copy volumes are L2- and
    // MALL-resident and the deeper loop's extra selects cost more: 256^3,
    // 17.4 against 18.3 ms).
    p.fwd_prefetch = p.fwd_pad_f32 ? 1 : 2;
    // Work order: with at least FWD_ORDER_MIN_ANGLES angles, blocks of 128
    // angles handed to the XCDs in turns of half a row band each, so that
    // all XCDs work on neighbouring detector rows of the same angles at a
    // time and the few z-slices those rays cross stay in the MALL; else
    // blocks of 8 with each XCD taking one eighth of the work in order.
    // 1500^3: 2.47-2.49 against 2.90 s (blocks of 64 or 256: 2.48 s);
    // 512^3 / 720 x 1024 x 768: 225 against 241 ms; 256^3 / 360 x 512^2:
    // 17.1 against 17.3 ms.
    if (g.n_angles >= FWD_ORDER_MIN_ANGLES) {
        p.fwd_angle_block = 128;
        p.fwd_xcd_chunk = 0;
    }
    // Where the padded copies stay 16-bit (volumes far larger than L2 and
    // the MALL), 8 angles per workgroup (512 threads), so that each line a
    // wave gathers serves twice as many waves of the same CU (1500^3, with
    // blocks of 16: 2.90 against 3.32 s; 16 angles: 3.16 s).  The FP32-copy
    // volumes keep 4 angles, which leave room for a fifth wave per SIMD
    // (256^3: 17.3 ms; 8 angles 17.7 ms, 16 angles 23.4 ms; 512^3 with
    // blocks of 128: 225 ms, 8 angles 243 ms).
    if (!p.fwd_pad_f32) p.fwd_wave_angles = 8;
    // Tuning override: KCT_FWD_PREFETCH selects how many segments ahead the
    // forward loop gathers (0, 1 or 2).
    if (const char *e = std::getenv("KCT_FWD_PREFETCH")) {
        const int d = std::atoi(e);
        if (d >= 0 && d <= 2) p.fwd_prefetch = d;
    }
    // Tuning override: the forward wave's patch width in detector columns.
    if (const char *e = std::getenv("KCT_FWD_LANES_U")) {
        const int lu = std::atoi(e);
        if (lu == 16 || lu == 32 || lu == 64) p.fwd_lane_u = lu;
    }
    // Tuning override: KCT_FWD_PAD_F32=0 keeps 16-bit padded copies.
    if (const char *e = std::getenv("KCT_FWD_PAD_F32")) p.fwd_pad_f32 = std::atoi(e) != 0;
    // Tuning override: angles per forward workgroup (1, 4, or 8 in a
    // workgroup of 512 threads).
    if (const char *e = std::getenv("KCT_FWD_WAVE_ANGLES")) {
        const int wa = std::atoi(e);
        if (wa == 1 || wa == 4 || wa == 8 || wa == 16) p.fwd_wave_angles = wa;
    }
    // Tuning override: angles per block of the forward work order (a power
    // of two, 4 to 4096).
    if (const char *e = std::getenv("KCT_FWD_ANGLE_BLOCK")) {
        const int ab = std::atoi(e);
        if (ab >= 4 && ab <= 4096 && (ab & (ab - 1)) == 0) p.fwd_angle_block = ab;
    }
    if (p.fwd_angle_block < p.fwd_wave_angles) p.fwd_angle_block = p.fwd_wave_angles;
    // Tuning override: logical tiles an XCD takes per turn (-1: one eighth
    // of all, in order; 0: half a row band; N > 0: N).
    if (const char *e = std::getenv("KCT_FWD_XCD_CHUNK")) p.fwd_xcd_chunk = std::max(-1LL, std::atoll(e));
}

} // namespace kct

using namespace kct;

extern "C" {

const char *kct_version(void) { return "kct 0.1 (gfx950)"; }

const char *kct_last_error(void) { return g_last_error.c_str(); }

const char *kct_status_str(kct_status s)
{
    switch (s) {
    case KCT_OK: return "ok";
    case KCT_E_INVALID_ARG: return "invalid argument";
    case KCT_E_GEOMETRY: return "unsupported geometry";
    case KCT_E_DTYPE: return "unsupported storage type";
    case KCT_E_OOM: return "out of device memory";
    case KCT_E_BUDGET: return "buffer too small";
    case KCT_E_DEVICE: return "device error";
    case KCT_E_NONFINITE: return "non-finite value";
    case KCT_E_STATE: return "invalid state";
    }
    return "unknown status";
}

kct_status kct_plan_create(const kct_geometry *geom, int device, kct_plan **out)
{
    g_last_error.clear();
    if (!out) return fail(KCT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    kct_status s = validate(geom);
    if (s != KCT_OK) return s;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(KCT_E_DEVICE, "no such HIP device");
    kct_plan *p = new (std::nothrow) kct_plan();
    if (!p) return fail(KCT_E_OOM, "host allocation failed");
    p->device = device;
    p->geom = *geom;
    p->angles.assign(geom->angles, geom->angles + geom->n_angles);
    p->geom.angles = p->angles.data();
    build_tables(*p);
    s = choose_bwd_shape(*p);
    if (s != KCT_OK) {
        delete p;
        return s;
    }
    choose_fwd_shape(*p);
    DeviceGuard dg(device);
    if (!dg.ok) {
        delete p;
        return fail(KCT_E_DEVICE, "hipSetDevice failed");
    }
    resolve_scratch(device);
    // 1/v per detector row.  The central row of an odd detector (v = 0) gets
    // 1e300 instead of infinity: z/v then maps a voxel with z0 <= 0 < z1 to an
    // interval covering every ray parameter in (0, 1) and excludes the others,
    // which is the half-open voxel rule for a ray inside the plane z = 0.
    std::vector<double> invv(geom->nv);
    for (int iv = 0; iv < geom->nv; ++iv) {
        const double v = (iv - p->gp.cv) * geom->dv;
        invv[iv] = v != 0.0 ? 1.0 / v : 1.0e300;
    }
    s = check_hip(hipMalloc(&p->d_tab, sizeof(AngleGeo) * geom->n_angles), "plan table allocation");
    if (s == KCT_OK) s = check_hip(hipMalloc(&p->d_invv, sizeof(double) * geom->nv), "plan table allocation");
    if (s == KCT_OK) s = check_hip(hipMalloc(&p->d_err, sizeof(int)), "plan flag allocation");
    if (s == KCT_OK)
        s = check_hip(hipMemcpy(p->d_tab, p->host_tab.data(), sizeof(AngleGeo) * geom->n_angles,
                                hipMemcpyHostToDevice), "plan table upload");
    if (s == KCT_OK)
        s = check_hip(hipMemcpy(p->d_invv, invv.data(), sizeof(double) * geom->nv, hipMemcpyHostToDevice),
                      "plan table upload");
    if (s == KCT_OK) s = check_hip(hipMemset(p->d_err, 0, sizeof(int)), "plan flag reset");
    if (s == KCT_OK)
        s = check_hip(hipMalloc(&p->d_dlen, sizeof(float) * size_t(geom->nu) * size_t(geom->nv)),
                      "plan table allocation");
    // The tables are used from any stream: build them on a private stream and
    // wait for that stream only (work the caller has in flight on other
    // streams, such as other requests' iterations, is not waited for).
    hipStream_t ts = nullptr;
    if (s == KCT_OK) s = check_hip(hipStreamCreateWithFlags(&ts, hipStreamNonBlocking), "plan stream creation");
    if (s == KCT_OK) s = launch_ray_lengths(*p, ts);
    if (s == KCT_OK) s = check_hip(hipStreamSynchronize(ts), "plan table build");
    if (ts) (void)hipStreamDestroy(ts);
    // Partial volumes of the angle-split back projection (small volumes
    // only, at most 16 x 2^18 floats without the KCT_BWD_SPLIT override), so
    // that kct_backproject only enqueues.
    if (s == KCT_OK && bwd_split_floats(*p) > 0) {
        const size_t need = sizeof(float) * size_t(bwd_split_floats(*p));
        s = check_hip(hipMalloc(&p->d_split, need), "partial volume allocation");
        if (s == KCT_OK) p->split_bytes = need;
    }
    if (s != KCT_OK) {
        kct_plan_destroy(p);
        return s;
    }
    *out = p;
    return KCT_OK;
}

kct_status kct_plan_reserve(kct_plan *p, int32_t vol_dtype)
{
    g_last_error.clear();
    if (!p) return fail(KCT_E_INVALID_ARG, "plan is NULL");
    if (!dtype_ok(vol_dtype)) return fail(KCT_E_DTYPE, "unknown storage type");
    const size_t need = size_t(2 * p->pad.vox) * dtype_size(fwd_pad_dtype(*p, vol_dtype));
    if (p->pad_bytes >= need) return KCT_OK;
    DeviceGuard dg(p->device);
    // The old copies may still be read by enqueued forward projections.
    if (p->d_pad) {
        kct_status s = check_hip(hipDeviceSynchronize(), "wait before replacing the padded copies");
        if (s != KCT_OK) return s;
        (void)hipFree(p->d_pad);
    }
    p->d_pad = nullptr;
    p->pad_bytes = 0;
    kct_status s = check_hip(hipMalloc(&p->d_pad, need), "padded volume allocation");
    if (s != KCT_OK) return s;
    p->pad_bytes = need;
    return KCT_OK;
}

kct_status kct_plan_check(kct_plan *p, void *stream)
{
    g_last_error.clear();
    if (!p) return fail(KCT_E_INVALID_ARG, "plan is NULL");
    DeviceGuard dg(p->device);
    kct_status s = check_hip(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "stream synchronisation");
    if (s != KCT_OK) return s;
    int v = 0;
    s = check_hip(hipMemcpy(&v, p->d_err, sizeof(int), hipMemcpyDeviceToHost), "error flag read");
    if (s != KCT_OK) return s;
    if (v == 0) return KCT_OK;
    s = check_hip(hipMemset(p->d_err, 0, sizeof(int)), "error flag reset");
    if (s != KCT_OK) return s;
    return fail(KCT_E_GEOMETRY, std::string("a back projection met a voxel footprint wider than the plan's bound (") +
                                    ((v & 1) ? "tile patch" : "") + ((v & 3) == 3 ? ", " : "") +
                                    ((v & 2) ? "voxel columns" : "") + "): its sums are truncated");
}

kct_status kct_plan_destroy(kct_plan *p)
{
    if (!p) return KCT_OK;
    DeviceGuard dg(p->device);
    if (p->d_tab) (void)hipFree(p->d_tab);
    if (p->d_invv) (void)hipFree(p->d_invv);
    if (p->d_dlen) (void)hipFree(p->d_dlen);
    if (p->d_err) (void)hipFree(p->d_err);
    if (p->d_pad) (void)hipFree(p->d_pad);
    if (p->d_split) (void)hipFree(p->d_split);
    delete p;
    return KCT_OK;
}

kct_status kct_plan_device_bytes(const kct_plan *p, size_t *bytes)
{
    if (!p || !bytes) return fail(KCT_E_INVALID_ARG, "NULL argument");
    *bytes = sizeof(AngleGeo) * p->gp.na + sizeof(double) * p->gp.nv + sizeof(float) * size_t(p->gp.nv) * p->gp.nu +
             sizeof(int) + p->pad_bytes + p->split_bytes;
    return KCT_OK;
}

kct_status kct_forward(kct_plan *p, const void *d_vol, int32_t vol_dtype, void *d_proj, int32_t proj_dtype,
                       void *stream)
{
    g_last_error.clear();
    if (!p || !d_vol || !d_proj) return fail(KCT_E_INVALID_ARG, "NULL argument");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(KCT_E_DTYPE, "unknown storage type");
    const int pdt = fwd_pad_dtype(*p, vol_dtype);
    const size_t need = size_t(2 * p->pad.vox) * dtype_size(pdt);
    if (p->pad_bytes < need)
        return fail(KCT_E_BUDGET, "the plan holds no padded copies for this volume storage type: call "
                                  "kct_plan_reserve(plan, vol_dtype) first");
    DeviceGuard dg(p->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    kct_status s = launch_pad_volume_as(*p, d_vol, vol_dtype, pdt, p->d_pad, st);
    if (s != KCT_OK) return s;
    Epilogue ep;
    return launch_forward(*p, p->d_pad, pdt, d_proj, proj_dtype, ep, st);
}

kct_status kct_forward_noalloc(kct_plan *p, const void *d_vol, int32_t vol_dtype, void *d_proj, int32_t proj_dtype,
                               void *stream)
{
    g_last_error.clear();
    if (!p || !d_vol || !d_proj) return fail(KCT_E_INVALID_ARG, "NULL argument");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(KCT_E_DTYPE, "unknown storage type");
    const int pdt = fwd_pad_dtype(*p, vol_dtype);
    const size_t need = size_t(2 * p->pad.vox) * dtype_size(pdt);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(KCT_E_BUDGET, "the padded volume copies (" + std::to_string(need) + " bytes) exceed the " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte static scratch of "
                                      "kct_forward_noalloc: use kct_plan_reserve and kct_forward");
    void *pad = scratch_address(p->device);
    if (!pad) return fail(KCT_E_DEVICE, "the static scratch's device address could not be resolved");
    DeviceGuard dg(p->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // The pad kernel writes every element of both copies, border included, so
    // nothing left by an earlier call is read.
    kct_status s = launch_pad_volume_as(*p, d_vol, vol_dtype, pdt, pad, st);
    if (s != KCT_OK) return s;
    Epilogue ep;
    return launch_forward(*p, pad, pdt, d_proj, proj_dtype, ep, st);
}

kct_status kct_backproject(kct_plan *p, const void *d_proj, int32_t proj_dtype, void *d_vol, int32_t vol_dtype,
                           void *stream)
{
    g_last_error.clear();
    if (!p || !d_vol || !d_proj) return fail(KCT_E_INVALID_ARG, "NULL argument");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(KCT_E_DTYPE, "unknown storage type");
    DeviceGuard dg(p->device);
    Epilogue ep;
    // Partial volumes of the angle-split back projection (small volumes),
    // allocated with the plan.
    ep.split = p->d_split;
    return launch_backward(*p, d_proj, proj_dtype, d_vol, vol_dtype, ep, static_cast<hipStream_t>(stream));
}

kct_status kct_backproject_interp(kct_plan *p, const void *d_proj, int32_t proj_dtype, void *d_vol, int32_t vol_dtype,
                                  void *stream)
{
    g_last_error.clear();
    if (!p || !d_vol || !d_proj) return fail(KCT_E_INVALID_ARG, "NULL argument");
    if (!dtype_ok(vol_dtype) || !dtype_ok(proj_dtype)) return fail(KCT_E_DTYPE, "unknown storage type");
    DeviceGuard dg(p->device);
    Epilogue ep;
    return launch_interp_backward(*p, d_proj, proj_dtype, d_vol, vol_dtype, ep, static_cast<hipStream_t>(stream));
}

// Test hooks, declared in kct.h.
int kct_debug_bwd_shape_geom(const kct_geometry *geom, int *kz, int *ncmax, int *pw, int *ph)
{
    kct_status s = validate(geom);
    if (s != KCT_OK) return s;
    Plan p;
    p.geom = *geom;
    p.angles.assign(geom->angles, geom->angles + geom->n_angles);
    p.geom.angles = p.angles.data();
    build_tables(p);
    s = choose_bwd_shape(p);
    if (s != KCT_OK) return s;
    if (kz) *kz = p.bwd_kz;
    if (ncmax) *ncmax = p.bwd_ncmax;
    if (pw) *pw = p.bwd_pw;
    if (ph) *ph = p.bwd_ph;
    return KCT_OK;
}

int kct_debug_fwd_shape_geom(const kct_geometry *geom, int *lane_u, int *wave_angles, int *angle_block, int *pad_f32)
{
    kct_status s = validate(geom);
    if (s != KCT_OK) return s;
    Plan p;
    p.geom = *geom;
    p.angles.assign(geom->angles, geom->angles + geom->n_angles);
    p.geom.angles = p.angles.data();
    build_tables(p);
    choose_fwd_shape(p);
    if (lane_u) *lane_u = p.fwd_lane_u;
    if (wave_angles) *wave_angles = p.fwd_wave_angles;
    if (angle_block) *angle_block = p.fwd_angle_block;
    if (pad_f32) *pad_f32 = p.fwd_pad_f32 ? 1 : 0;
    return KCT_OK;
}

int kct_debug_bwd_mode_geom(const kct_geometry *geom, int *split, int *rays)
{
    kct_status s = validate(geom);
    if (s != KCT_OK) return s;
    Plan p;
    p.geom = *geom;
    p.angles.assign(geom->angles, geom->angles + geom->n_angles);
    p.geom.angles = p.angles.data();
    build_tables(p);
    s = choose_bwd_shape(p);
    if (s != KCT_OK) return s;
    if (split) *split = std::min(p.bwd_asplit, p.gp.na);
    if (rays) *rays = p.bwd_rays ? 1 : 0;
    return KCT_OK;
}

void kct_debug_bwd_mode(const kct_plan *p, int *split, int *rays)
{
    if (!p) return;
    if (split) *split = std::min(p->bwd_asplit, p->gp.na);
    if (rays) *rays = p->bwd_rays ? 1 : 0;
}

void kct_debug_bwd_shape(const kct_plan *p, int *kz, int *ncmax, int *pw, int *ph)
{
    if (!p) return;
    if (kz) *kz = p->bwd_kz;
    if (ncmax) *ncmax = p->bwd_ncmax;
    if (pw) *pw = p->bwd_pw;
    if (ph) *ph = p->bwd_ph;
}

} // extern "C"
