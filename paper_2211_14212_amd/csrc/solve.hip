// Solver drivers: workspace layout and the per-iteration kernel sequences of
// CGLS, LSQR, LSMR and hybrid LSQR (paper Sec. 2.1 and Sec. 2.2).  Every
// step is enqueued on the caller's stream; the Krylov scalars live in device
// FP64 memory, so the host never waits inside the loop.
//
// Per iteration (-> marks a fused epilogue):
//   CGLS    pad(p); q = A p -> ||q||^2; alpha; r += -alpha q -> ||r||^2;
//           s = A^T r - lam^2 (x + alpha p) -> ||s||^2; beta;
//           x += alpha p, p = s + beta p -> ||p||^2
//   LSQR    pad(V); U = A V / alpha - (alpha/beta) U -> ||U||^2; beta;
//           V = A^T U / beta - (beta/alpha) V -> ||V||^2; alpha, rotations;
//           x += (phi/rho) w, w = V/alpha - (theta/rho) w
//   LSMR    as LSQR, then hbar, x, h updates in one pass
//   hybrid  as LSQR's bidiagonalisation with V_k kept; at the end the small
//           projected Tikhonov problem is solved on the device and x = V_k y
//   IRN-TV  (Sec. 2.3.1) outer k: weights L from x (L = I at k = 0), restart
//           r1 = b - A x, r2 = -lam L D x, s = A^T r1 + lam D^T L r2, p = s;
//           inner CGLS on [A; lam L D]: q1 = A p -> ||q1||^2 and
//           ||lam L D p||^2; alpha; r1 -= alpha q1; r2 -= alpha lam L D p;
//           s = A^T r1 + lam D^T L r2 -> ||s||^2; beta; x, p updates
//   AB-GMRES (Sec. 2.1.4) z = B V_j; V_{j+1} = A z; modified Gram-Schmidt
//           against V_1..V_j (dot, scalar, axpy per vector); normalise;
//           Givens update of H and of the residual.  At the end
//           x = B (sum_i y_i V_i).  BA-GMRES: t = A V_j; V_{j+1} = B t; ...;
//           x = sum_i y_i V_i.
//   SIRT / OS-SART (Sec. 3) per subset s: r_s = b_s - A_s x -> ||r_s||^2;
//           r_s *= W; v = A_s^T r_s; x += lam V_s v.  The angles are
//           permuted once so that every subset is a contiguous block, and the
//           projectors run on a view of the plan holding that block.
//   fLSQR-TV (Sec. 2.3.2) weights L from x (L = I at k = 0); r = A^T u_k;
//           r = E^T r; t = K^+ r (inner CG); V_k = L D t, orthonormalised
//           against V_1..V_{k-1}; r = D^T L V_k; t = K^+ r; Z_k = E t;
//           u_{k+1} = A Z_k orthonormalised against u_1..u_k (column k of
//           M); projected Tikhonov solve of (M_k, beta1 e1); x = x0 + Z_k y.

#include "flsqr.hpp"
#include "gmres.hpp"
#include "krylov.hpp"
#include "sart.hpp"

#include <cmath>
#include <cstdlib>
#include <new>
#include <vector>

namespace kct {

namespace {

constexpr size_t ALIGN = 256;

size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t scal = 0, pa = 0, pb = 0, pc = 0, stage = 0, gk = 0, work = 0, coef = 0, pad = 0, bsplit = 0;
    size_t v[6] = {0, 0, 0, 0, 0, 0};
    size_t total = 0;
    int64_t nparts = 0;
};

bool solver_ok(int s) { return s >= KCT_CGLS && s <= KCT_HYBRID_FLSQR_TV; }

bool is_sart(int s) { return s == KCT_SIRT || s == KCT_OS_SART; }

bool is_gmres(int s) { return s == KCT_AB_GMRES || s == KCT_BA_GMRES; }

kct_status check_params(const kct_solve_params *prm)
{
    if (!prm) return fail(KCT_E_INVALID_ARG, "params is NULL");
    if (!solver_ok(prm->solver)) return fail(KCT_E_INVALID_ARG, "unknown solver");
    if (prm->solver == KCT_IRN_TV_CGLS) {
        if (prm->tv_outer < 1 || prm->tv_inner < 1 || int64_t(prm->tv_outer) * prm->tv_inner > 100000)
            return fail(KCT_E_INVALID_ARG, "IRN-TV needs tv_outer >= 1 and tv_inner >= 1");
        if (!(prm->tv_eps > 0.0) || !std::isfinite(prm->tv_eps)) return fail(KCT_E_INVALID_ARG, "tv_eps must be > 0");
    }
    if (prm->solver == KCT_HYBRID_FLSQR_TV) {
        if (prm->tv_inner < 1 || prm->tv_inner > 10000)
            return fail(KCT_E_INVALID_ARG, "fLSQR-TV needs tv_inner >= 1 CG steps per pseudoinverse");
        if (prm->tv_outer != 0) return fail(KCT_E_INVALID_ARG, "fLSQR-TV takes no tv_outer (n_iter iterations)");
        if (!(prm->tv_eps > 0.0) || !std::isfinite(prm->tv_eps)) return fail(KCT_E_INVALID_ARG, "tv_eps must be > 0");
        if (prm->vec_dtype != KCT_F32) return fail(KCT_E_DTYPE, "fLSQR-TV stores its vectors in FP32");
    }
    if (prm->n_iter < 0 || prm->n_iter > 100000) return fail(KCT_E_INVALID_ARG, "n_iter out of range");
    if (!(prm->lambda >= 0.0) || !std::isfinite(prm->lambda)) return fail(KCT_E_INVALID_ARG, "lambda must be >= 0");
    if (!dtype_ok(prm->vec_dtype)) return fail(KCT_E_DTYPE, "unknown vector storage type");
    if (prm->backprojector != KCT_BP_MATCHED) {
        if (prm->backprojector != KCT_BP_INTERP) return fail(KCT_E_INVALID_ARG, "unknown back projector");
        if (!is_gmres(prm->solver))
            return fail(KCT_E_INVALID_ARG, "only AB- and BA-GMRES take an unmatched back projector");
    }
    if (prm->flags & ~(KCT_FLAG_STOP_ON_RESIDUAL_INCREASE | KCT_FLAG_EXPLICIT_RESIDUAL | KCT_FLAG_X0_GIVEN))
        return fail(KCT_E_INVALID_ARG, "unknown flags");
    if (prm->flags & KCT_FLAG_X0_GIVEN) {
        const int sv = prm->solver;
        if (sv != KCT_CGLS && sv != KCT_LSQR && sv != KCT_LSMR && !is_sart(sv))
            return fail(KCT_E_INVALID_ARG, "a given x0 is for CGLS, LSQR, LSMR, SIRT and OS-SART");
        if ((sv == KCT_LSQR || sv == KCT_LSMR) && prm->lambda != 0.0)
            return fail(KCT_E_INVALID_ARG, "LSQR and LSMR start from a given x0 only without damping");
    }
    if (prm->reserved != 0) return fail(KCT_E_INVALID_ARG, "reserved must be 0");
    if ((prm->flags & (KCT_FLAG_STOP_ON_RESIDUAL_INCREASE | KCT_FLAG_EXPLICIT_RESIDUAL)) &&
        prm->solver != KCT_CGLS && prm->solver != KCT_LSQR &&
        prm->solver != KCT_LSMR)
        return fail(KCT_E_INVALID_ARG, "explicit residuals and the stop rule are for CGLS, LSQR and LSMR");
    if (is_sart(prm->solver)) {
        if (!(prm->lambda > 0.0 && prm->lambda < 2.0))
            return fail(KCT_E_INVALID_ARG, "SIRT / OS-SART need a relaxation lambda in (0, 2)");
        if (prm->vec_dtype != KCT_F32) return fail(KCT_E_DTYPE, "SIRT / OS-SART run in FP32");
        if (prm->solver == KCT_OS_SART && prm->n_subsets < 1)
            return fail(KCT_E_INVALID_ARG, "OS-SART needs n_subsets >= 1");
        if (prm->solver == KCT_SIRT && prm->n_subsets > 1)
            return fail(KCT_E_INVALID_ARG, "SIRT takes no subsets (use OS-SART)");
    } else if (prm->n_subsets != 0) {
        return fail(KCT_E_INVALID_ARG, "n_subsets is for OS-SART only");
    }
    if (is_gmres(prm->solver)) {
        if (prm->lambda != 0.0) return fail(KCT_E_INVALID_ARG, "AB-/BA-GMRES solve the undamped problem (lambda 0)");
        // Unit basis vectors have entries near 1/sqrt(n): below FP16's normal range.
        if (prm->vec_dtype == KCT_F16) return fail(KCT_E_DTYPE, "AB-/BA-GMRES store their basis in FP32 or BF16");
    }
    if (prm->lambda_rule != KCT_LAMBDA_FIXED) {
        if (prm->lambda_rule != KCT_LAMBDA_GCV && prm->lambda_rule != KCT_LAMBDA_DP)
            return fail(KCT_E_INVALID_ARG, "unknown lambda rule");
        if (prm->solver != KCT_HYBRID_LSQR && prm->solver != KCT_HYBRID_FLSQR_TV)
            return fail(KCT_E_INVALID_ARG, "only hybrid LSQR and fLSQR-TV choose lambda during the iterations");
        if (prm->lambda_rule == KCT_LAMBDA_DP && !(prm->noise_level > 0.0 && std::isfinite(prm->noise_level)))
            return fail(KCT_E_INVALID_ARG, "the discrepancy principle needs a noise level > 0");
    }
    return KCT_OK;
}

kct_status check_params_plan(const Plan &p, const kct_solve_params &prm)
{
    if (prm.solver == KCT_OS_SART && prm.n_subsets > p.gp.na)
        return fail(KCT_E_INVALID_ARG, "OS-SART has more subsets than angles");
    return KCT_OK;
}

Layout layout(const Plan &p, const kct_solve_params &prm)
{
    Layout L;
    const int64_t N = p.n_ray(), M = p.n_vox();
    const size_t vt = dtype_size(prm.vec_dtype);
    Plan one = p; // OS-SART's subset views project with one angle per workgroup
    one.fwd_wave_angles = 1;
    L.nparts = std::max<int64_t>({fwd_num_groups(p), fwd_num_groups(one), bwd_num_groups(p), ibp_num_groups(p),
                                  int64_t(VEC_GROUPS), int64_t(GM_GROUPS)});
    size_t o = 0;
    L.scal = o; o += up(sizeof(double) * S_COUNT);
    L.pa = o; o += up(sizeof(double) * L.nparts);
    L.pb = o; o += up(sizeof(double) * L.nparts);
    L.pc = o; o += up(sizeof(double) * L.nparts);
    L.stage = o; o += up(sizeof(double) * 3 * 256);
    const bool expl = prm.flags & (KCT_FLAG_STOP_ON_RESIDUAL_INCREASE | KCT_FLAG_EXPLICIT_RESIDUAL);
    // The stop rule projects x itself (FP32), so its padded copy needs FP32;
    // so do 16-bit vectors when the plan widens them for the forward.
    const size_t pad_elem = std::max({vt, dtype_size(fwd_pad_dtype(p, prm.vec_dtype)), expl ? size_t(4) : size_t(0)});
    L.pad = o; o += up(size_t(2 * p.pad.vox) * pad_elem);
    L.bsplit = o; o += up(sizeof(float) * size_t(bwd_split_floats(p))); // partial volumes (small volumes)
    const int k = prm.n_iter;
    switch (prm.solver) {
    case KCT_CGLS:
        L.v[0] = o; o += up(size_t(N) * vt); // r
        L.v[1] = o; o += up(size_t(N) * vt); // q
        L.v[2] = o; o += up(size_t(M) * vt); // p
        L.v[3] = o; o += up(size_t(M) * vt); // s
        break;
    case KCT_LSQR:
        L.v[0] = o; o += up(size_t(N) * vt); // U
        L.v[1] = o; o += up(size_t(M) * vt); // V
        L.v[2] = o; o += up(size_t(M) * 4);  // w
        break;
    case KCT_LSMR:
        L.v[0] = o; o += up(size_t(N) * vt); // U
        L.v[1] = o; o += up(size_t(M) * vt); // V
        L.v[2] = o; o += up(size_t(M) * 4);  // h
        L.v[3] = o; o += up(size_t(M) * 4);  // hbar
        break;
    case KCT_HYBRID_LSQR:
        L.v[0] = o; o += up(size_t(N) * vt);                 // U
        L.v[1] = o; o += up(size_t(M) * vt * size_t(k + 1)); // basis V_1..V_{k+1}
        L.gk = o; o += up(sizeof(double) * (2 * size_t(k) + 4));
        // QR of [B_k; lam I] (fixed lambda) or W, Q, sigma, c, y of the SVD (GCV, DP).
        L.work = o; o += up(sizeof(double) * ((2 * size_t(k) + 1) * (size_t(k) + 1) + 4 * size_t(k) + 8));
        L.coef = o; o += up(sizeof(double) * (size_t(k) + 1));
        break;
    case KCT_AB_GMRES:
    case KCT_BA_GMRES: {
        const bool ab = prm.solver == KCT_AB_GMRES;
        const int64_t nb = ab ? N : M, nt = ab ? M : N;
        L.v[0] = o; o += up(size_t(nb) * vt * size_t(k + 1)); // basis V_1..V_{k+1}
        L.v[1] = o; o += up(size_t(nt) * vt);                 // B V_j (AB) or A V_j (BA)
        if (ab) { L.v[2] = o; o += up(size_t(N) * 4); }       // sum_i y_i V_i before the last B
        L.gk = o; o += up(sizeof(double) * (size_t(k) + 1) * size_t(std::max(k, 1))); // H
        L.work = o; o += up(sizeof(double) * (3 * size_t(k) + 2));                   // cs, sn, g
        L.coef = o; o += up(sizeof(double) * (size_t(k) + 1));
        break;
    }
    case KCT_SIRT:
    case KCT_OS_SART: {
        const int m = prm.solver == KCT_SIRT ? 1 : prm.n_subsets;
        L.v[0] = o; o += up(size_t(N) * 4);              // residual r (permuted angle order)
        L.v[1] = o; o += up(size_t(M) * 4);              // A_s^T (W r_s)
        L.v[2] = o; o += up(size_t(N) * 4);              // W
        L.v[3] = o; o += up(size_t(M) * 4 * size_t(m));  // V_1..V_m
        if (m > 1) {
            L.v[4] = o; o += up(size_t(N) * 4);          // b in the permuted angle order
            L.work = o; o += up(sizeof(AngleGeo) * size_t(p.gp.na));
        }
        break;
    }
    case KCT_HYBRID_FLSQR_TV: {
        const size_t kk = size_t(std::max(k, 1));
        L.v[0] = o; o += up(size_t(N) * 4 * std::max<size_t>(k + 1, 2)); // u_1..u_{k+1} (u_2 holds A 1 at first)
        L.v[1] = o; o += up(size_t(M) * 4 * 3 * kk);                     // V_1..V_k, gradient space
        L.v[2] = o; o += up(size_t(M) * 4 * kk);                         // Z_1..Z_k
        L.v[3] = o; o += up(size_t(M) * 4);                              // g = A^T A 1
        L.v[4] = o; o += up(size_t(M) * 4 * 2 + size_t(M) * 8 * 4);      // t, r (FP32); inner CG t, r, p, q (FP64)
        L.v[5] = o; o += up(size_t(M) * 4);                              // L weights
        L.gk = o; o += up(sizeof(double) * (kk + 1) * kk * 2);           // M ((k+1) x k), T (k x k)
        L.work = o; o += up(sizeof(double) * ((2 * kk + 1) * (kk + 1) + 5 * kk + 10));
        L.coef = o; o += up(sizeof(double) * (kk + 1));
        break;
    }
    case KCT_IRN_TV_CGLS:
        L.v[0] = o; o += up(size_t(N) * vt);    // r1
        L.v[1] = o; o += up(size_t(N) * vt);    // q1
        L.v[2] = o; o += up(size_t(M) * vt);    // p
        L.v[3] = o; o += up(size_t(M) * vt);    // s
        L.v[4] = o; o += up(size_t(M) * 4 * 3); // r2 (gradient space, FP32)
        L.v[5] = o; o += up(size_t(M) * 4);     // L weights
        break;
    }
    if (expl) {
        L.v[4] = o; o += up(size_t(M) * 4); // x of the previous iteration
        L.v[5] = o; o += up(size_t(N) * 4); // b - A x_k
    }
    L.total = o;
    return L;
}

} // namespace

} // namespace kct

using namespace kct;

struct kct_state {
    kct_plan *plan = nullptr;
    kct_solve_params prm{};
    const float *b = nullptr;
    float *x = nullptr;
    char *ws = nullptr;
    double *hist = nullptr;
    hipStream_t st = nullptr;
    Layout L;
    int enqueued = 0;
    bool started = false;
    bool finalized = false;
    int total = 0; // iterations to run (IRN-TV: outer * inner)
    // SIRT / OS-SART: the plan restricted to each subset's block of the
    // permuted angles (views: they share the plan's device buffers), the
    // first angle of each block (and the angle count at the end).
    std::vector<kct::Plan> sub;
    std::vector<int> sub_a0;
    // CGLS, opt-in: one iteration captured into a HIP graph and replayed per
    // step (every kernel argument is the same from the second iteration on).
    bool use_graph = false;
    bool graph_failed = false;
    hipGraphExec_t graph = nullptr;

    double *S() const { return reinterpret_cast<double *>(ws + L.scal); }
    double *pa() const { return reinterpret_cast<double *>(ws + L.pa); }
    double *pb() const { return reinterpret_cast<double *>(ws + L.pb); }
    double *pc() const { return reinterpret_cast<double *>(ws + L.pc); }
    double *stage(int i) const { return reinterpret_cast<double *>(ws + L.stage) + 256 * i; }
    void *pad() const { return ws + L.pad; }
    void *v(int i) const { return ws + L.v[i]; }
    int vt() const { return prm.vec_dtype; }
    int64_t N() const { return plan->n_ray(); }
    int64_t M() const { return plan->n_vox(); }
};

namespace {

#define KCT_TRY(expr)                                                                                              \
    do {                                                                                                           \
        kct_status s_ = (expr);                                                                                    \
        if (s_ != KCT_OK) return s_;                                                                               \
    } while (0)

Reduced red(const kct_state &s, const double *parts, int64_t n, int slot)
{
    return reduce_for_scalar(parts, n, s.stage(slot), s.st);
}

// The back projector with this state's partial-volume buffer (used when the
// plan splits the angles of a small volume over several workgroups).
kct_status backward_into(kct_state &s, Plan &p, const void *proj, int pdt, void *vol, int vdt, Epilogue ep)
{
    ep.split = reinterpret_cast<float *>(s.ws + s.L.bsplit);
    ep.err_scal = s.S(); // a footprint overflow becomes history code 4
    return launch_backward(p, proj, pdt, vol, vdt, ep, s.st);
}

kct_status forward_into(kct_state &s, const void *vol, void *proj, const Epilogue &ep)
{
    Plan &p = *s.plan;
    const int pdt = fwd_pad_dtype(p, s.vt());
    KCT_TRY(launch_pad_volume_as(p, vol, s.vt(), pdt, s.pad(), s.st));
    return launch_forward(p, s.pad(), pdt, proj, s.vt(), ep, s.st);
}

// ---------------------------------------------------------------- CGLS
bool x0_given(const kct_state &s) { return s.prm.flags & KCT_FLAG_X0_GIVEN; }

// r = b - A x (x FP32; its padded copy in the forward's padding storage),
// in place on r = b.
kct_status residual_from_x(kct_state &s, void *r, double *partials)
{
    Plan &p = *s.plan;
    const int pdt = fwd_pad_dtype(p, s.vt());
    KCT_TRY(launch_pad_volume_as(p, s.x, KCT_F32, pdt, s.pad(), s.st));
    Epilogue ef;
    ef.c[0] = -1.0;
    ef.c[1] = 1.0;
    ef.in1 = r;
    ef.partials = partials;
    return launch_forward(p, s.pad(), pdt, r, s.vt(), ef, s.st);
}

kct_status cgls_init(kct_state &s)
{
    Plan &p = *s.plan;
    if (!x0_given(s)) KCT_TRY(vk_fill(s.x, KCT_F32, s.M(), 0.f, s.st));
    KCT_TRY(vk_scale(s.b, KCT_F32, s.v(0), s.vt(), s.N(), nullptr, -1, nullptr, s.st)); // r = b
    Epilogue ep;
    ep.partials = s.pa();
    if (x0_given(s)) { // r = b - A x0, s = A^T r - lam^2 x0
        KCT_TRY(residual_from_x(s, s.v(0), nullptr));
        if (s.prm.lambda != 0.0) {
            ep.c[2] = -s.prm.lambda * s.prm.lambda;
            ep.in2 = s.x;
        }
    }
    KCT_TRY(backward_into(s, p, s.v(0), s.vt(), s.v(2), s.vt(), ep)); // p = A^T r
    return sk_cgls_init(s.S(), red(s, s.pa(), bwd_num_groups(p), 0), s.prm.lambda, s.prm.n_iter, s.st);
}

kct_status cgls_iter(kct_state &s)
{
    Plan &p = *s.plan;
    const bool damped = s.prm.lambda != 0.0;
    Epilogue ef;
    ef.scal = s.S();
    ef.partials = s.pa();
    KCT_TRY(forward_into(s, s.v(2), s.v(1), ef)); // q = A p
    const Reduced rq = red(s, s.pa(), fwd_num_groups(p), 0);
    // ||p||^2 comes from the previous volume update; at the first step p = s
    // and the scalar kernel uses gamma instead.
    const Reduced rp = (damped && s.enqueued > 0) ? red(s, s.pc(), vk_groups(s.M()), 1) : Reduced{nullptr, 0};
    KCT_TRY(sk_cgls_alpha(s.S(), rq, rp, s.st));
    KCT_TRY(vk_axpy_proj(s.v(0), s.v(1), s.vt(), s.N(), s.S(), s.pb(), s.st)); // r -= alpha q
    Epilogue eb;
    eb.scal = s.S();
    eb.coef_idx = S_B0;
    eb.partials = s.pa();
    if (damped) {
        eb.in2 = s.x;
        eb.in3 = s.v(2);
    }
    KCT_TRY(backward_into(s, p, s.v(0), s.vt(), s.v(3), s.vt(), eb)); // s = A^T r - lam^2 x'
    KCT_TRY(sk_cgls_beta(s.S(), red(s, s.pa(), bwd_num_groups(p), 0), red(s, s.pb(), vk_groups(s.N()), 2),
                         s.hist, s.st));
    return vk_cgls_vol(s.x, s.v(2), s.v(3), s.vt(), s.M(), s.S(), s.pc(), s.st);
}

// ------------------------------------------------------- Golub-Kahan start
kct_status gk_init(kct_state &s, void *V, double *gk)
{
    Plan &p = *s.plan;
    const bool x0 = x0_given(s); // LSQR / LSMR without damping: Golub-Kahan from b - A x0
    if (!x0) KCT_TRY(vk_fill(s.x, KCT_F32, s.M(), 0.f, s.st));
    KCT_TRY(vk_scale(s.b, KCT_F32, s.v(0), s.vt(), s.N(), nullptr, -1, x0 ? nullptr : s.pa(), s.st)); // U = b
    if (x0) KCT_TRY(residual_from_x(s, s.v(0), s.pa())); // U = b - A x0
    const Reduced ru = red(s, s.pa(), x0 ? fwd_num_groups(p) : vk_groups(s.N()), 0);
    // LSQR's damping; hybrid LSQR with a lambda rule recurs undamped quantities.
    const double lam = s.prm.lambda_rule == KCT_LAMBDA_FIXED ? s.prm.lambda : 0.0;
    KCT_TRY(sk_gk_init1(s.S(), ru, lam, s.prm.n_iter, s.st));
    Epilogue eb;
    eb.scal = s.S();
    eb.coef_idx = S_B0; // V = A^T U / beta_1
    eb.partials = s.pa();
    KCT_TRY(backward_into(s, p, s.v(0), s.vt(), V, s.vt(), eb));
    return sk_gk_init2(s.S(), red(s, s.pa(), bwd_num_groups(p), 0), gk, s.st);
}

// One bidiagonalisation step: U from V_in, then V_out from U (in place when equal).
kct_status gk_step(kct_state &s, void *V_in, void *V_out)
{
    Plan &p = *s.plan;
    Epilogue ef;
    ef.scal = s.S();
    ef.coef_idx = S_F0;
    ef.in1 = s.v(0);
    ef.partials = s.pa();
    KCT_TRY(forward_into(s, V_in, s.v(0), ef));
    KCT_TRY(sk_gk_beta(s.S(), red(s, s.pa(), fwd_num_groups(p), 0), s.st));
    Epilogue eb;
    eb.scal = s.S();
    eb.coef_idx = S_B0;
    eb.in1 = V_in;
    eb.partials = s.pa();
    return backward_into(s, p, s.v(0), s.vt(), V_out, s.vt(), eb);
}

kct_status lsqr_init(kct_state &s)
{
    KCT_TRY(gk_init(s, s.v(1), nullptr));
    return vk_scale(s.v(1), s.vt(), s.v(2), KCT_F32, s.M(), s.S(), S_V0, nullptr, s.st); // w = V / alpha_1
}

kct_status lsqr_iter(kct_state &s)
{
    KCT_TRY(gk_step(s, s.v(1), s.v(1)));
    KCT_TRY(sk_lsqr_alpha(s.S(), red(s, s.pa(), bwd_num_groups(*s.plan), 0), s.hist, nullptr, s.st));
    return vk_lsqr_vol(s.x, static_cast<float *>(s.v(2)), s.v(1), s.vt(), s.M(), s.S(), s.st);
}

kct_status lsmr_init(kct_state &s)
{
    KCT_TRY(gk_init(s, s.v(1), nullptr));
    KCT_TRY(vk_scale(s.v(1), s.vt(), s.v(2), KCT_F32, s.M(), s.S(), S_V0, nullptr, s.st)); // h = V / alpha_1
    return vk_fill(s.v(3), KCT_F32, s.M(), 0.f, s.st);                                     // hbar = 0
}

kct_status lsmr_iter(kct_state &s)
{
    KCT_TRY(gk_step(s, s.v(1), s.v(1)));
    KCT_TRY(sk_lsmr_alpha(s.S(), red(s, s.pa(), bwd_num_groups(*s.plan), 0), s.hist, s.st));
    return vk_lsmr_vol(s.x, static_cast<float *>(s.v(2)), static_cast<float *>(s.v(3)), s.v(1), s.vt(), s.M(),
                       s.S(), s.st);
}

void *basis_slot(kct_state &s, int i)
{
    return static_cast<char *>(s.v(1)) + size_t(i) * size_t(s.M()) * dtype_size(s.vt());
}

double *gk_arr(kct_state &s) { return reinterpret_cast<double *>(s.ws + s.L.gk); }

kct_status hybrid_init(kct_state &s) { return gk_init(s, basis_slot(s, 0), gk_arr(s)); }

kct_status hybrid_iter(kct_state &s)
{
    const int k = s.enqueued;
    KCT_TRY(gk_step(s, basis_slot(s, k), basis_slot(s, k + 1)));
    KCT_TRY(sk_lsqr_alpha(s.S(), red(s, s.pa(), bwd_num_groups(*s.plan), 0), s.hist, gk_arr(s), s.st));
    if (s.prm.lambda_rule == KCT_LAMBDA_FIXED) return KCT_OK;
    // lambda_k for this iteration: SVD of B_k, the rule's search, y_k.
    double *work = reinterpret_cast<double *>(s.ws + s.L.work);
    double *coef = reinterpret_cast<double *>(s.ws + s.L.coef);
    return sk_hybrid_choose(s.S(), gk_arr(s), work, coef, s.hist, s.prm.lambda_rule, s.prm.noise_level, s.st);
}

kct_status hybrid_finish(kct_state &s)
{
    double *work = reinterpret_cast<double *>(s.ws + s.L.work);
    double *coef = reinterpret_cast<double *>(s.ws + s.L.coef);
    // With GCV or DP the last iteration already left y_k in coef.
    if (s.prm.lambda_rule == KCT_LAMBDA_FIXED) KCT_TRY(sk_hybrid_solve(s.S(), gk_arr(s), work, coef, s.st));
    return vk_combine(s.x, s.v(1), s.vt(), s.M(), coef, s.S(), s.st);
}

// ---------------------------------------------------------------- IRN-TV
float *tv_r2(kct_state &s) { return static_cast<float *>(s.v(4)); }
float *tv_w(kct_state &s) { return static_cast<float *>(s.v(5)); }

kct_status irn_begin_outer(kct_state &s, int outer)
{
    Plan &p = *s.plan;
    const double lam = s.prm.lambda;
    if (outer == 0) {
        KCT_TRY(vk_fill(tv_w(s), KCT_F32, s.M(), 1.f, s.st)); // L = I
    } else {
        KCT_TRY(tv_weights(p, s.x, tv_w(s), s.prm.tv_eps, s.st));
    }
    KCT_TRY(vk_scale(s.b, KCT_F32, s.v(0), s.vt(), s.N(), nullptr, -1, nullptr, s.st)); // r1 = b
    if (outer > 0) {
        // r1 = b - A x, r2 = -lam L D x (x is FP32; its padded copy is in the
        // forward's padding storage)
        const int pdt = fwd_pad_dtype(p, s.vt());
        KCT_TRY(launch_pad_volume_as(p, s.x, KCT_F32, pdt, s.pad(), s.st));
        Epilogue ef;
        ef.c[0] = -1.0;
        ef.c[1] = 1.0;
        ef.in1 = s.v(0);
        KCT_TRY(launch_forward(p, s.pad(), pdt, s.v(0), s.vt(), ef, s.st));
        KCT_TRY(tv_grad_store(p, s.x, KCT_F32, tv_w(s), tv_r2(s), nullptr, -1, -lam, false, s.st));
    } else {
        KCT_TRY(vk_fill(tv_r2(s), KCT_F32, 3 * s.M(), 0.f, s.st));
    }
    Epilogue eb;
    KCT_TRY(backward_into(s, p, s.v(0), s.vt(), s.v(3), s.vt(), eb)); // s = A^T r1
    KCT_TRY(tv_adjoint_add(p, s.v(3), s.vt(), tv_r2(s), tv_w(s), lam, nullptr, s.pa(), s.st));
    KCT_TRY(vk_scale(s.v(3), s.vt(), s.v(2), s.vt(), s.M(), nullptr, -1, nullptr, s.st)); // p = s
    return sk_tv_restart(s.S(), red(s, s.pa(), tv_num_groups(s.M()), 0), outer == 0, s.total, s.prm.lambda, s.st);
}

kct_status irn_init(kct_state &s)
{
    KCT_TRY(vk_fill(s.x, KCT_F32, s.M(), 0.f, s.st));
    return irn_begin_outer(s, 0);
}

kct_status irn_iter(kct_state &s)
{
    Plan &p = *s.plan;
    const double lam = s.prm.lambda;
    Epilogue ef;
    ef.scal = s.S();
    ef.partials = s.pa();
    KCT_TRY(forward_into(s, s.v(2), s.v(1), ef)); // q1 = A p
    KCT_TRY(tv_grad_norm(p, s.v(2), s.vt(), tv_w(s), lam, s.S(), s.pb(), s.st));
    KCT_TRY(sk_tv_alpha(s.S(), red(s, s.pa(), fwd_num_groups(p), 0), red(s, s.pb(), tv_num_groups(s.M()), 1), lam,
                        s.st));
    KCT_TRY(vk_axpy_proj(s.v(0), s.v(1), s.vt(), s.N(), s.S(), s.pc(), s.st));            // r1 -= alpha q1
    KCT_TRY(tv_grad_store(p, s.v(2), s.vt(), tv_w(s), tv_r2(s), s.S(), S_V3, 0.0, true, s.st)); // r2
    Epilogue eb;
    eb.scal = s.S();
    KCT_TRY(backward_into(s, p, s.v(0), s.vt(), s.v(3), s.vt(), eb)); // s = A^T r1
    KCT_TRY(tv_adjoint_add(p, s.v(3), s.vt(), tv_r2(s), tv_w(s), lam, s.S(), s.pa(), s.st));
    KCT_TRY(sk_cgls_beta(s.S(), red(s, s.pa(), tv_num_groups(s.M()), 0), red(s, s.pc(), vk_groups(s.N()), 2),
                         s.hist, s.st));
    KCT_TRY(vk_cgls_vol(s.x, s.v(2), s.v(3), s.vt(), s.M(), s.S(), s.pb(), s.st));
    const int done = s.enqueued + 1;
    if (done % s.prm.tv_inner == 0 && done < s.total) KCT_TRY(irn_begin_outer(s, done / s.prm.tv_inner));
    return KCT_OK;
}

// ---------------------------------------------------------------- AB-/BA-GMRES
bool gm_ab(const kct_state &s) { return s.prm.solver == KCT_AB_GMRES; }
int64_t gm_n(const kct_state &s) { return gm_ab(s) ? s.N() : s.M(); } // basis vector length
int gm_ldh(const kct_state &s) { return s.prm.n_iter + 1; }
double *gm_H(kct_state &s) { return reinterpret_cast<double *>(s.ws + s.L.gk); }
double *gm_cs(kct_state &s) { return reinterpret_cast<double *>(s.ws + s.L.work); }
double *gm_sn(kct_state &s) { return gm_cs(s) + s.prm.n_iter; }
double *gm_g(kct_state &s) { return gm_sn(s) + s.prm.n_iter; }
void *gm_V(kct_state &s, int i) { return static_cast<char *>(s.v(0)) + size_t(i) * size_t(gm_n(s)) * dtype_size(s.vt()); }

// y = B x with the solver's back projector; the partial sums of y^2 per
// workgroup go to ep.partials.
kct_status apply_B(kct_state &s, const void *proj, int pdt, void *vol, int vdt, const Epilogue &ep)
{
    if (s.prm.backprojector == KCT_BP_INTERP) return launch_interp_backward(*s.plan, proj, pdt, vol, vdt, ep, s.st);
    return backward_into(s, *s.plan, proj, pdt, vol, vdt, ep);
}

int64_t B_groups(const kct_state &s)
{
    return s.prm.backprojector == KCT_BP_INTERP ? ibp_num_groups(*s.plan) : bwd_num_groups(*s.plan);
}

kct_status gm_init(kct_state &s)
{
    KCT_TRY(vk_fill(s.x, KCT_F32, s.M(), 0.f, s.st));
    void *V0 = gm_V(s, 0);
    Reduced r0;
    if (gm_ab(s)) { // r0 = b
        KCT_TRY(vk_scale(s.b, KCT_F32, V0, s.vt(), s.N(), nullptr, -1, s.pa(), s.st));
        r0 = red(s, s.pa(), vk_groups(s.N()), 0);
    } else { // r0 = B b
        Epilogue ep;
        ep.partials = s.pa();
        KCT_TRY(apply_B(s, s.b, KCT_F32, V0, s.vt(), ep));
        r0 = red(s, s.pa(), B_groups(s), 0);
    }
    KCT_TRY(gm_sc_init(s.S(), r0.ptr, r0.n, gm_g(s), s.prm.n_iter, s.st));
    return gm_scale(V0, s.vt(), gm_n(s), s.S(), S_V0, s.st);
}

kct_status gm_iter(kct_state &s)
{
    const int j = s.enqueued, ldh = gm_ldh(s);
    const int64_t n = gm_n(s);
    void *Vj = gm_V(s, j), *W = gm_V(s, j + 1);
    Epilogue plain;
    if (gm_ab(s)) {
        KCT_TRY(apply_B(s, Vj, s.vt(), s.v(1), s.vt(), plain)); // z = B V_j
        KCT_TRY(forward_into(s, s.v(1), W, plain));             // W = A z
    } else {
        KCT_TRY(forward_into(s, Vj, s.v(1), plain));            // t = A V_j
        KCT_TRY(apply_B(s, s.v(1), s.vt(), W, s.vt(), plain)); // W = B t
    }
    for (int i = 0; i <= j; ++i) { // modified Gram-Schmidt
        KCT_TRY(gm_dot(W, gm_V(s, i), s.vt(), n, s.pa(), s.st));
        const Reduced h = red(s, s.pa(), gm_num_groups(n), 0);
        KCT_TRY(gm_sc_h(s.S(), h.ptr, h.n, gm_H(s), i, j, ldh, s.st));
        KCT_TRY(gm_axpy(W, gm_V(s, i), s.vt(), n, s.S(), S_P0, s.st));
    }
    KCT_TRY(gm_dot(W, W, s.vt(), n, s.pa(), s.st));
    const Reduced w2 = red(s, s.pa(), gm_num_groups(n), 0);
    KCT_TRY(gm_sc_norm(s.S(), w2.ptr, w2.n, gm_H(s), j, ldh, s.st));
    KCT_TRY(gm_scale(W, s.vt(), n, s.S(), S_V0, s.st));
    return gm_sc_givens(s.S(), gm_H(s), gm_cs(s), gm_sn(s), gm_g(s), j, ldh, s.hist, s.st);
}

kct_status gm_finish(kct_state &s)
{
    double *coef = reinterpret_cast<double *>(s.ws + s.L.coef);
    KCT_TRY(gm_sc_solve(s.S(), gm_H(s), gm_g(s), coef, gm_ldh(s), s.st));
    if (!gm_ab(s)) return vk_combine(s.x, s.v(0), s.vt(), s.M(), coef, s.S(), s.st);
    float *z = static_cast<float *>(s.v(2));
    KCT_TRY(vk_combine(z, s.v(0), s.vt(), s.N(), coef, s.S(), s.st)); // sum_i y_i V_i
    Epilogue plain;
    return apply_B(s, z, KCT_F32, s.x, KCT_F32, plain);                 // x = B (...)
}

// ---------------------------------------------------------------- SIRT / OS-SART
int sa_m(const kct_state &s) { return s.prm.solver == KCT_SIRT ? 1 : s.prm.n_subsets; }
float *sa_r(kct_state &s) { return static_cast<float *>(s.v(0)); }
float *sa_v(kct_state &s) { return static_cast<float *>(s.v(1)); }
float *sa_W(kct_state &s) { return static_cast<float *>(s.v(2)); }
float *sa_V(kct_state &s, int k) { return static_cast<float *>(s.v(3)) + size_t(k) * size_t(s.M()); }
const float *sa_b(kct_state &s) { return sa_m(s) > 1 ? static_cast<const float *>(s.v(4)) : s.b; }
size_t sa_off(const kct_state &s, int k) { return size_t(s.sub_a0[k]) * size_t(s.plan->gp.nv) * s.plan->gp.nu; }

// The host side of SART's set-up: subset k holds the angles a = k, k + m, ...,
// laid out as the k-th contiguous block of the permuted order (its table in
// the workspace when m > 1); s.sub[k] is the plan restricted to that block.
void sa_views(kct_state &s)
{
    Plan &p = *s.plan;
    const int m = sa_m(s), na = p.gp.na;
    s.sub_a0.clear();
    for (int k = 0; k <= m; ++k) s.sub_a0.push_back(k < m ? sa_block_start(k, na, m) : na);
    AngleGeo *tab = m > 1 ? reinterpret_cast<AngleGeo *>(s.ws + s.L.work) : p.d_tab;
    s.sub.assign(m, p);
    for (int k = 0; k < m; ++k) {
        Plan &v = s.sub[k];
        v.d_tab = tab + s.sub_a0[k];
        v.gp.na = s.sub_a0[k + 1] - s.sub_a0[k];
        v.bwd_fp_angles = std::min(v.bwd_fp_angles, v.gp.na);
        // A block's neighbouring angles lie m angles apart, so workgroups
        // that trace one patch at 4 of them share no voxel lines: the
        // forward uses the one-angle shape (46.8 against 42.3 ms per
        // 10-subset iteration on 256^3 / 360 x 512^2).
        if (m > 1) v.fwd_wave_angles = 1;
        // A subset too small for the large-plan work order takes the small
        // one (a block of 128 angles would hold mostly empty tiles).
        if (v.gp.na < FWD_ORDER_MIN_ANGLES && v.fwd_angle_block > 8) {
            v.fwd_angle_block = std::max(8, v.fwd_wave_angles);
            v.fwd_xcd_chunk = -1;
        }
    }
}

kct_status sa_init(kct_state &s)
{
    Plan &p = *s.plan;
    const int m = sa_m(s), na = p.gp.na;
    sa_views(s);
    if (m > 1)
        KCT_TRY(sa_permute(reinterpret_cast<AngleGeo *>(s.ws + s.L.work), p.d_tab, static_cast<float *>(s.v(4)),
                           s.b, na, int64_t(p.gp.nv) * p.gp.nu, m, s.st));
    Epilogue plain;
    // W = 1 / (A 1): every block's rays through a volume of ones.
    KCT_TRY(vk_fill(sa_v(s), KCT_F32, s.M(), 1.f, s.st));
    KCT_TRY(launch_pad_volume(p, sa_v(s), KCT_F32, s.pad(), s.st));
    for (int k = 0; k < m; ++k)
        KCT_TRY(launch_forward(s.sub[k], s.pad(), KCT_F32, sa_W(s) + sa_off(s, k), KCT_F32, plain, s.st));
    KCT_TRY(sa_inv_nz(sa_W(s), s.N(), s.st));
    // V_k = 1 / (A_k^T 1).
    KCT_TRY(vk_fill(sa_r(s), KCT_F32, s.N(), 1.f, s.st));
    for (int k = 0; k < m; ++k)
        KCT_TRY(backward_into(s, s.sub[k], sa_r(s) + sa_off(s, k), KCT_F32, sa_V(s, k), KCT_F32, plain));
    KCT_TRY(sa_inv_nz(sa_V(s, 0), int64_t(m) * s.M(), s.st));
    if (!x0_given(s)) KCT_TRY(vk_fill(s.x, KCT_F32, s.M(), 0.f, s.st));
    return sa_sc_init(s.S(), s.prm.n_iter, s.prm.lambda, s.st);
}

kct_status sa_iter(kct_state &s)
{
    Plan &p = *s.plan;
    const int m = sa_m(s);
    for (int k = 0; k < m; ++k) {
        Plan &v = s.sub[k];
        float *r = sa_r(s) + sa_off(s, k);
        const int64_t nk = int64_t(v.gp.na) * v.gp.nv * v.gp.nu;
        Epilogue ef; // r_k = b_k - A_k x, with ||r_k||^2 per workgroup
        ef.c[0] = -1.0;
        ef.c[1] = 1.0;
        ef.in1 = sa_b(s) + sa_off(s, k);
        ef.partials = s.pa();
        KCT_TRY(launch_pad_volume(p, s.x, KCT_F32, s.pad(), s.st));
        KCT_TRY(launch_forward(v, s.pad(), KCT_F32, r, KCT_F32, ef, s.st));
        const Reduced rr = red(s, s.pa(), fwd_num_groups(v), 0);
        KCT_TRY(sa_sc_res(s.S(), rr.ptr, rr.n, s.hist, k == 0, k == m - 1, s.st));
        KCT_TRY(sa_mul(r, sa_W(s) + sa_off(s, k), nk, s.st));
        Epilogue plain;
        KCT_TRY(backward_into(s, v, r, KCT_F32, sa_v(s), KCT_F32, plain));
        KCT_TRY(sa_update_x(s.x, sa_v(s), sa_V(s, k), s.M(), s.S(), s.st));
    }
    return KCT_OK;
}

// ---------------------------------------------------------------- fLSQR-TV
int fl_K(const kct_state &s) { return std::max(s.prm.n_iter, 1); }
int fl_ldm(const kct_state &s) { return s.prm.n_iter + 1; }
float *fl_U(kct_state &s, int i) { return static_cast<float *>(s.v(0)) + size_t(i) * size_t(s.N()); }
float *fl_V(kct_state &s, int i) { return static_cast<float *>(s.v(1)) + size_t(i) * 3 * size_t(s.M()); }
float *fl_Z(kct_state &s, int i) { return static_cast<float *>(s.v(2)) + size_t(i) * size_t(s.M()); }
float *fl_g(kct_state &s) { return static_cast<float *>(s.v(3)); }
float *fl_tmp(kct_state &s, int i) { return static_cast<float *>(s.v(4)) + size_t(i) * size_t(s.M()); }
float *fl_w(kct_state &s) { return static_cast<float *>(s.v(5)); }
// The inner CG's FP64 vectors, after the two FP32 volumes of v(4).
double *fl_d(kct_state &s, int i)
{
    return reinterpret_cast<double *>(static_cast<float *>(s.v(4)) + 2 * size_t(s.M())) + size_t(i) * size_t(s.M());
}
double *fl_Mat(kct_state &s) { return reinterpret_cast<double *>(s.ws + s.L.gk); }
double *fl_T(kct_state &s) { return fl_Mat(s) + size_t(fl_ldm(s)) * size_t(fl_K(s)); }

kct_status fl_init(kct_state &s)
{
    Plan &p = *s.plan;
    const int64_t N = s.N(), M = s.M();
    float *a = fl_U(s, 1); // A 1, until the first iteration writes u_2
    KCT_TRY(vk_fill(fl_tmp(s, 0), KCT_F32, M, 1.f, s.st));
    Epilogue ef;
    ef.partials = s.pa();
    KCT_TRY(forward_into(s, fl_tmp(s, 0), a, ef)); // a = A 1 -> ||a||^2
    const Reduced rca = red(s, s.pa(), fwd_num_groups(p), 0);
    KCT_TRY(gm_dot(a, s.b, KCT_F32, N, s.pb(), s.st)); // a^T b
    KCT_TRY(fl_sc_init(s.S(), rca, red(s, s.pb(), gm_num_groups(N), 1), s.prm.n_iter, s.prm.lambda, s.st));
    KCT_TRY(fl_fill_s(s.x, M, s.S(), S_FL_C0, s.st)); // x = x0
    Epilogue eb;
    KCT_TRY(backward_into(s, p, a, KCT_F32, fl_g(s), KCT_F32, eb)); // g = A^T a
    KCT_TRY(fl_bbar(fl_U(s, 0), s.b, a, N, s.S(), s.pa(), s.st));        // bbar = b - c0 a -> ||bbar||^2
    KCT_TRY(fl_sc_beta1(s.S(), red(s, s.pa(), fl_groups(N), 0), s.st));
    return gm_scale(fl_U(s, 0), KCT_F32, N, s.S(), S_V0, s.st);
}

// t = K^+ r by tv_inner CG steps; the sums of r's entries and squares are in
// pa and pb (nparts each) from the kernel that produced r.
kct_status fl_cg(kct_state &s, int64_t nparts)
{
    Plan &p = *s.plan;
    const int64_t M = s.M();
    // The right-hand side arrives in fl_tmp(s, 1) (FP32); the result leaves in
    // fl_tmp(s, 0) (FP32); the CG itself runs in FP64.
    double *t = fl_d(s, 0), *r = fl_d(s, 1), *pv = fl_d(s, 2), *q = fl_d(s, 3);
    const int ng = fl_groups(M);
    KCT_TRY(fl_sc_cg_init(s.S(), red(s, s.pa(), nparts, 0), red(s, s.pb(), nparts, 1), M, s.st));
    KCT_TRY(fl_cg_dir(r, pv, t, fl_tmp(s, 1), M, s.S(), s.st));
    for (int it = 0; it < s.prm.tv_inner; ++it) {
        KCT_TRY(fl_lap(p, pv, fl_w(s), q, s.pa(), s.st));
        KCT_TRY(fl_sc_cg_alpha(s.S(), red(s, s.pa(), ng, 0), s.st));
        KCT_TRY(fl_cg_update(t, r, pv, q, M, s.S(), s.pa(), s.pb(), s.st));
        if (it + 1 == s.prm.tv_inner) break;
        KCT_TRY(fl_sc_cg_beta(s.S(), red(s, s.pa(), ng, 0), red(s, s.pb(), ng, 1), M, s.st));
        KCT_TRY(fl_cg_dir(r, pv, t, nullptr, M, s.S(), s.st));
    }
    return fl_to_f32(fl_tmp(s, 0), t, M, s.st);
}

kct_status fl_iter(kct_state &s)
{
    Plan &p = *s.plan;
    const int k = s.enqueued, ldm = fl_ldm(s);
    const int64_t N = s.N(), M = s.M(), M3 = 3 * M;
    float *t = fl_tmp(s, 0), *r = fl_tmp(s, 1);
    if (k == 0) KCT_TRY(vk_fill(fl_w(s), KCT_F32, M, 1.f, s.st)); // L = I
    else KCT_TRY(tv_weights(p, s.x, fl_w(s), s.prm.tv_eps, s.st));
    // v = P^T A^T u_k = L D K^+ E^T A^T u_k.
    Epilogue eb;
    KCT_TRY(backward_into(s, p, fl_U(s, k), KCT_F32, r, KCT_F32, eb));
    KCT_TRY(fl_sum(r, M, s.pa(), s.st));
    KCT_TRY(fl_sc_ecoef(s.S(), red(s, s.pa(), fl_groups(M), 0), S_FL_E, s.st));
    KCT_TRY(fl_axpy_sum(r, fl_g(s), M, s.S(), S_FL_E, s.pa(), s.pb(), s.st));
    KCT_TRY(fl_cg(s, fl_groups(M)));
    float *Vk = fl_V(s, k);
    KCT_TRY(tv_grad_store(p, t, KCT_F32, fl_w(s), Vk, nullptr, -1, 1.0, false, s.st));
    for (int i = 0; i < k; ++i) { // modified Gram-Schmidt against v_1..v_{k-1}
        KCT_TRY(gm_dot(Vk, fl_V(s, i), KCT_F32, M3, s.pa(), s.st));
        const Reduced h = red(s, s.pa(), gm_num_groups(M3), 0);
        KCT_TRY(gm_sc_h(s.S(), h.ptr, h.n, fl_T(s), i, k, fl_K(s), s.st));
        KCT_TRY(gm_axpy(Vk, fl_V(s, i), KCT_F32, M3, s.S(), S_P0, s.st));
    }
    KCT_TRY(gm_dot(Vk, Vk, KCT_F32, M3, s.pa(), s.st));
    KCT_TRY(fl_sc_vnorm(s.S(), red(s, s.pa(), gm_num_groups(M3), 0), s.st));
    KCT_TRY(gm_scale(Vk, KCT_F32, M3, s.S(), S_V0, s.st));
    // z_k = P v_k = E K^+ D^T L v_k.
    KCT_TRY(fl_dtl(p, Vk, fl_w(s), r, s.pa(), s.pb(), s.st));
    KCT_TRY(fl_cg(s, fl_groups(M)));
    KCT_TRY(gm_dot(fl_g(s), t, KCT_F32, M, s.pa(), s.st));
    KCT_TRY(fl_sc_ecoef(s.S(), red(s, s.pa(), gm_num_groups(M), 0), S_FL_E, s.st));
    float *Zk = fl_Z(s, k);
    KCT_TRY(fl_shift(Zk, t, M, s.S(), S_FL_E, s.st));
    // u_{k+1}: A z_k orthonormalised against u_1..u_k, coefficients in column k of M.
    float *U1 = fl_U(s, k + 1);
    Epilogue ef;
    KCT_TRY(forward_into(s, Zk, U1, ef));
    for (int i = 0; i <= k; ++i) {
        KCT_TRY(gm_dot(U1, fl_U(s, i), KCT_F32, N, s.pa(), s.st));
        const Reduced h = red(s, s.pa(), gm_num_groups(N), 0);
        KCT_TRY(gm_sc_h(s.S(), h.ptr, h.n, fl_Mat(s), i, k, ldm, s.st));
        KCT_TRY(gm_axpy(U1, fl_U(s, i), KCT_F32, N, s.S(), S_P0, s.st));
    }
    KCT_TRY(gm_dot(U1, U1, KCT_F32, N, s.pa(), s.st));
    const Reduced u2 = red(s, s.pa(), gm_num_groups(N), 0);
    KCT_TRY(gm_sc_norm(s.S(), u2.ptr, u2.n, fl_Mat(s), k, ldm, s.st));
    KCT_TRY(gm_scale(U1, KCT_F32, N, s.S(), S_V0, s.st));
    // Projected Tikhonov solve with lambda_k, then x = x0 + Z_k y.
    double *work = reinterpret_cast<double *>(s.ws + s.L.work);
    double *coef = reinterpret_cast<double *>(s.ws + s.L.coef);
    KCT_TRY(fl_sc_hist(s.S(), fl_Mat(s), k, ldm, s.hist, s.st));
    KCT_TRY(sk_hybrid_choose_dense(s.S(), fl_Mat(s), ldm, work, coef, s.hist, s.prm.lambda_rule,
                                   s.prm.noise_level, s.st));
    return fl_combine(s.x, fl_Z(s, 0), M, coef, s.S(), s.st);
}

kct_status enqueue_init(kct_state &s)
{
    // S_ERR (one double) starts at 0: a fill kernel, not a memset, so that
    // the start can be captured into a graph.
    KCT_TRY(vk_fill(s.S() + S_ERR, KCT_F32, 2, 0.f, s.st));
    switch (s.prm.solver) {
    case KCT_CGLS: return cgls_init(s);
    case KCT_LSQR: return lsqr_init(s);
    case KCT_LSMR: return lsmr_init(s);
    case KCT_HYBRID_LSQR: return hybrid_init(s);
    case KCT_IRN_TV_CGLS: return irn_init(s);
    case KCT_AB_GMRES:
    case KCT_BA_GMRES: return gm_init(s);
    case KCT_SIRT:
    case KCT_OS_SART: return sa_init(s);
    case KCT_HYBRID_FLSQR_TV: return fl_init(s);
    }
    return fail(KCT_E_INVALID_ARG, "unknown solver");
}

kct_status solver_iter(kct_state &s);

// One iteration, with the explicit residual (and the stop rule) after it when asked.
kct_status enqueue_iter(kct_state &s)
{
    const bool stop = s.prm.flags & KCT_FLAG_STOP_ON_RESIDUAL_INCREASE;
    if (!stop && !(s.prm.flags & KCT_FLAG_EXPLICIT_RESIDUAL)) return solver_iter(s);
    Plan &p = *s.plan;
    float *xp = static_cast<float *>(s.v(4));
    if (stop) KCT_TRY(vk_save_x(s.x, xp, s.M(), s.S(), s.st));
    KCT_TRY(solver_iter(s));
    Epilogue ef; // b - A x_k, with partial sums of its square
    ef.c[0] = -1.0;
    ef.c[1] = 1.0;
    ef.in1 = s.b;
    ef.partials = s.pa();
    KCT_TRY(launch_pad_volume(p, s.x, KCT_F32, s.pad(), s.st));
    KCT_TRY(launch_forward(p, s.pad(), KCT_F32, s.v(5), KCT_F32, ef, s.st));
    KCT_TRY(sk_explicit(s.S(), red(s, s.pa(), fwd_num_groups(p), 0), s.hist, stop, s.st));
    return stop ? vk_restore_x(s.x, xp, s.M(), s.S(), s.st) : KCT_OK;
}

kct_status solver_iter(kct_state &s)
{
    switch (s.prm.solver) {
    case KCT_CGLS: return cgls_iter(s);
    case KCT_LSQR: return lsqr_iter(s);
    case KCT_LSMR: return lsmr_iter(s);
    case KCT_HYBRID_LSQR: return hybrid_iter(s);
    case KCT_IRN_TV_CGLS: return irn_iter(s);
    case KCT_AB_GMRES:
    case KCT_BA_GMRES: return gm_iter(s);
    case KCT_SIRT:
    case KCT_OS_SART: return sa_iter(s);
    case KCT_HYBRID_FLSQR_TV: return fl_iter(s);
    }
    return fail(KCT_E_INVALID_ARG, "unknown solver");
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(d);
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

} // namespace

extern "C" {

kct_status kct_solve_workspace_bytes(const kct_plan *plan, const kct_solve_params *params, size_t *bytes)
{
    if (!plan || !bytes) return fail(KCT_E_INVALID_ARG, "NULL argument");
    KCT_TRY(check_params(params));
    KCT_TRY(check_params_plan(*plan, *params));
    *bytes = layout(*plan, *params).total;
    return KCT_OK;
}

kct_status kct_state_create(kct_plan *plan, const kct_solve_params *params, const void *d_b, void *d_x,
                            void *d_ws, size_t ws_bytes, double *d_history, void *stream, kct_state **out)
{
    if (!out) return fail(KCT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!plan || !d_b || !d_x || !d_ws) return fail(KCT_E_INVALID_ARG, "NULL argument");
    KCT_TRY(check_params(params));
    KCT_TRY(check_params_plan(*plan, *params));
    const Layout L = layout(*plan, *params);
    if (ws_bytes < L.total) return fail(KCT_E_BUDGET, "workspace smaller than kct_solve_workspace_bytes");
    if (reinterpret_cast<uintptr_t>(d_ws) % ALIGN) return fail(KCT_E_INVALID_ARG, "workspace must be 256-byte aligned");
    kct_state *s = new (std::nothrow) kct_state();
    if (!s) return fail(KCT_E_OOM, "host allocation failed");
    s->plan = plan;
    s->prm = *params;
    s->b = static_cast<const float *>(d_b);
    s->x = static_cast<float *>(d_x);
    s->ws = static_cast<char *>(d_ws);
    s->hist = d_history;
    s->st = static_cast<hipStream_t>(stream);
    s->L = L;
    s->total = params->solver == KCT_IRN_TV_CGLS ? params->tv_outer * params->tv_inner : params->n_iter;
    // Opt-in (KCT_SOLVE_GRAPHS=1): CGLS replays one captured iteration.  It is
    // bitwise the enqueued run, but on 32^3 / 36 x 64^2 (8 launches per
    // iteration) a replay took 57 us against 51-53 us for direct launches,
    // so it is off by default.
    if (const char *e = std::getenv("KCT_SOLVE_GRAPHS"))
        s->use_graph = std::atoi(e) != 0 && params->solver == KCT_CGLS &&
                       !(params->flags & (KCT_FLAG_STOP_ON_RESIDUAL_INCREASE | KCT_FLAG_EXPLICIT_RESIDUAL));
    *out = s;
    return KCT_OK;
}

kct_status kct_state_resume(kct_plan *plan, const kct_solve_params *params, const void *d_b, void *d_x,
                            void *d_ws, size_t ws_bytes, double *d_history, void *stream, int32_t iters_done,
                            kct_state **out)
{
    if (out) *out = nullptr;
    kct_state *s = nullptr;
    KCT_TRY(kct_state_create(plan, params, d_b, d_x, d_ws, ws_bytes, d_history, stream, &s));
    if (iters_done < 0 || iters_done > s->total) {
        kct_state_destroy(s);
        return fail(KCT_E_INVALID_ARG, "iters_done outside 0..the run's iteration count");
    }
    // Host-side set-up only: the device state is already in the buffers.
    if (is_sart(s->prm.solver)) sa_views(*s);
    s->started = true;
    s->enqueued = iters_done;
    s->finalized = iters_done == s->total;
    *out = s;
    return KCT_OK;
}

// Capture one iteration of `s` on its stream into s.graph.  The captured
// launches do not run; the caller launches the graph.  False (and no graph)
// when the stream cannot be captured: the legacy default stream, or a stream
// the caller is already capturing.
static bool capture_iter(kct_state &s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s.st == nullptr || hipStreamIsCapturing(s.st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return false;
    }
    if (hipStreamBeginCapture(s.st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const kct_status e = solver_iter(s);
    hipGraph_t g = nullptr;
    const hipError_t he = hipStreamEndCapture(s.st, &g);
    bool ok = e == KCT_OK && he == hipSuccess && g != nullptr;
    if (ok) ok = hipGraphInstantiate(&s.graph, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        s.graph = nullptr;
        (void)hipGetLastError();
    }
    return ok;
}

kct_status kct_state_step(kct_state *s, int32_t n_steps)
{
    if (!s || n_steps < 0) return fail(KCT_E_INVALID_ARG, "bad state or step count");
    DevGuard dg(s->plan->device);
    if (!s->started) {
        KCT_TRY(enqueue_init(*s));
        s->started = true;
    }
    for (int i = 0; i < n_steps && s->enqueued < s->total; ++i) {
        // Opt-in: from the second iteration on, replay one captured
        // iteration.  Any failure to capture falls back to enqueueing the
        // kernels.
        if (s->use_graph && s->enqueued >= 1 && !s->graph_failed) {
            if (!s->graph && !capture_iter(*s)) s->graph_failed = true;
            if (s->graph) {
                KCT_TRY(check_hip(hipGraphLaunch(s->graph, s->st), "solver iteration graph launch"));
                ++s->enqueued;
                continue;
            }
        }
        KCT_TRY(enqueue_iter(*s));
        ++s->enqueued;
    }
    if (s->enqueued == s->total && !s->finalized) {
        if (s->prm.solver == KCT_HYBRID_LSQR) KCT_TRY(hybrid_finish(*s));
        if (is_gmres(s->prm.solver)) KCT_TRY(gm_finish(*s));
        s->finalized = true;
    }
    return KCT_OK;
}

kct_status kct_state_progress(const kct_state *s, int32_t *iters, int32_t *finished)
{
    if (!s) return fail(KCT_E_INVALID_ARG, "state is NULL");
    if (iters) *iters = s->enqueued;
    if (finished) *finished = s->finalized ? 1 : 0;
    return KCT_OK;
}

kct_status kct_state_destroy(kct_state *s)
{
    if (s && s->graph) {
        DevGuard dg(s->plan->device);
        (void)hipGraphExecDestroy(s->graph);
    }
    delete s;
    return KCT_OK;
}

kct_status kct_solve(kct_plan *plan, const kct_solve_params *params, const void *d_b, void *d_x, void *d_ws,
                     size_t ws_bytes, double *d_history, void *stream)
{
    kct_state *s = nullptr;
    KCT_TRY(kct_state_create(plan, params, d_b, d_x, d_ws, ws_bytes, d_history, stream, &s));
    const kct_status r = kct_state_step(s, s->total);
    kct_state_destroy(s);
    return r;
}

} // extern "C"
