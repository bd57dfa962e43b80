/*
 * Oracle: FP64 Siddon ray tracing for circular cone-beam CT.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU oracle that checks
 * the GPU library.  It shares no code with the GPU path, and only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  The product path never calls it.
 *
 * What it computes (paper, Sec. 1, eq. (original_pbm)): the system
 * matrix A of A x + e = b, with N = detector pixels x angles rows and
 * M = voxels columns.  A is never stored; each row is traced on the fly.
 * Entry a_ij is the length (mm) of the segment of ray i inside voxel j
 * (Siddon's exact radiological path; the paper leaves the discretisation to
 * its toolbox, so this reading is stated in the design notes).
 *
 * Geometry (the paper gives none; this is the convention both sides
 * implement independently):
 *   voxel (i,j,k) = [X0+i*vx, X0+(i+1)*vx) x [Y0+j*vy, ...) x [Z0+k*vz, ...)
 *   with X0 = ox - nx*vx/2 (same for y, z); layout x[k][j][i].
 *   source      s = (DSO cos t, DSO sin t, 0)
 *   det. centre c = s + DSD (-cos t, -sin t, 0)
 *   e_u = (-sin t, cos t, 0), e_v = (0, 0, 1)
 *   pixel (iu,iv) centre = c + (iu-(nu-1)/2) du e_u + (iv-(nv-1)/2) dv e_v
 *   one ray per pixel: the segment from s to the pixel centre.
 *   projections y[a][iv][iu].
 *
 * Traversal (merged-parameter form of Siddon 1985): parametrise the ray as
 * p(t) = s + t d, d = pixel - s, t in [0,1].  Clip t to the volume box, list
 * every axis-plane crossing strictly inside the clipped range, merge the three
 * increasing lists, and give each consecutive pair of parameters the voxel that
 * contains the pair's midpoint; its length is (t1 - t0) |d|.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    double ox, oy, oz;
    int32_t nu, nv;
    double du, dv;
    double dso, dsd;
    int32_t na;
    const double *angles; /* radians, na entries */
} ora_geom;

/* One ray's crossing lists and output segments live in caller-provided scratch. */
typedef struct {
    double *tx, *ty, *tz, *tm; /* per-axis crossings and merged list */
    int64_t *idx;              /* voxel linear index per segment */
    double *len;               /* segment length (mm) */
} ora_scratch;

static int axis_range(double p0, double d, double lo, double hi, double *tmin, double *tmax)
{
    /* Parameter interval in which p0 + t d lies inside [lo, hi). */
    if (d == 0.0) {
        if (p0 < lo || p0 >= hi) return 0;
        *tmin = -INFINITY;
        *tmax = INFINITY;
        return 1;
    }
    double a = (lo - p0) / d, b = (hi - p0) / d;
    *tmin = a < b ? a : b;
    *tmax = a < b ? b : a;
    return 1;
}

/* Crossings of planes lo + m*v (m = 0..n) with t strictly inside (t0, t1), increasing. */
static int axis_crossings(double p0, double d, double lo, double v, int n, double t0, double t1, double *out)
{
    int c = 0;
    if (d == 0.0) return 0;
    if (d > 0.0) {
        for (int m = 0; m <= n; ++m) {
            double t = (lo + m * v - p0) / d;
            if (t > t0 && t < t1) out[c++] = t;
        }
    } else {
        for (int m = n; m >= 0; --m) {
            double t = (lo + m * v - p0) / d;
            if (t > t0 && t < t1) out[c++] = t;
        }
    }
    return c;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Trace ray (a, iv, iu).  Returns the number of segments written to s->idx / s->len. */
static int trace_ray(const ora_geom *g, int a, int iv, int iu, ora_scratch *s)
{
    double th = g->angles[a];
    double ct = cos(th), st = sin(th);
    double sx = g->dso * ct, sy = g->dso * st, sz = 0.0;
    double cx = sx - g->dsd * ct, cy = sy - g->dsd * st, cz = 0.0;
    double u = (iu - 0.5 * (g->nu - 1)) * g->du;
    double v = (iv - 0.5 * (g->nv - 1)) * g->dv;
    double px = cx - u * st, py = cy + u * ct, pz = cz + v;
    double dx = px - sx, dy = py - sy, dz = pz - sz;
    double dn = sqrt(dx * dx + dy * dy + dz * dz);

    double X0 = g->ox - 0.5 * g->nx * g->vx, X1 = X0 + g->nx * g->vx;
    double Y0 = g->oy - 0.5 * g->ny * g->vy, Y1 = Y0 + g->ny * g->vy;
    double Z0 = g->oz - 0.5 * g->nz * g->vz, Z1 = Z0 + g->nz * g->vz;

    double a0, a1, b0, b1, c0, c1;
    if (!axis_range(sx, dx, X0, X1, &a0, &a1)) return 0;
    if (!axis_range(sy, dy, Y0, Y1, &b0, &b1)) return 0;
    if (!axis_range(sz, dz, Z0, Z1, &c0, &c1)) return 0;
    double tmin = 0.0, tmax = 1.0;
    if (a0 > tmin) tmin = a0;
    if (b0 > tmin) tmin = b0;
    if (c0 > tmin) tmin = c0;
    if (a1 < tmax) tmax = a1;
    if (b1 < tmax) tmax = b1;
    if (c1 < tmax) tmax = c1;
    if (!(tmin < tmax)) return 0;

    int nxc = axis_crossings(sx, dx, X0, g->vx, g->nx, tmin, tmax, s->tx);
    int nyc = axis_crossings(sy, dy, Y0, g->vy, g->ny, tmin, tmax, s->ty);
    int nzc = axis_crossings(sz, dz, Z0, g->vz, g->nz, tmin, tmax, s->tz);

    /* Three-way merge of the increasing lists, bracketed by the end points. */
    int m = 0, ix = 0, iy = 0, iz = 0;
    s->tm[m++] = tmin;
    while (ix < nxc || iy < nyc || iz < nzc) {
        double bx = ix < nxc ? s->tx[ix] : INFINITY;
        double by = iy < nyc ? s->ty[iy] : INFINITY;
        double bz = iz < nzc ? s->tz[iz] : INFINITY;
        if (bx <= by && bx <= bz) s->tm[m++] = s->tx[ix++];
        else if (by <= bz) s->tm[m++] = s->ty[iy++];
        else s->tm[m++] = s->tz[iz++];
    }
    s->tm[m++] = tmax;

    int nseg = 0;
    for (int q = 0; q + 1 < m; ++q) {
        double t0 = s->tm[q], t1 = s->tm[q + 1];
        if (!(t1 > t0)) continue;
        double tc = 0.5 * (t0 + t1);
        int i = clampi((int)floor((sx + tc * dx - X0) / g->vx), 0, g->nx - 1);
        int j = clampi((int)floor((sy + tc * dy - Y0) / g->vy), 0, g->ny - 1);
        int k = clampi((int)floor((sz + tc * dz - Z0) / g->vz), 0, g->nz - 1);
        s->idx[nseg] = ((int64_t)k * g->ny + j) * g->nx + i;
        s->len[nseg] = (t1 - t0) * dn;
        ++nseg;
    }
    return nseg;
}

static int scratch_alloc(const ora_geom *g, ora_scratch *s)
{
    size_t n = (size_t)g->nx + g->ny + g->nz + 8;
    s->tx = malloc(n * sizeof(double));
    s->ty = malloc(n * sizeof(double));
    s->tz = malloc(n * sizeof(double));
    s->tm = malloc(3 * n * sizeof(double));
    s->idx = malloc(3 * n * sizeof(int64_t));
    s->len = malloc(3 * n * sizeof(double));
    return s->tx && s->ty && s->tz && s->tm && s->idx && s->len;
}

static void scratch_free(ora_scratch *s)
{
    free(s->tx); free(s->ty); free(s->tz); free(s->tm); free(s->idx); free(s->len);
}

/* y = A x.  x: [nz][ny][nx] FP64, y: [na][nv][nu] FP64.  Returns 0 on success. */
int ora_forward(const ora_geom *g, const double *x, double *y)
{
    int64_t nray = (int64_t)g->na * g->nv * g->nu;
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        ora_scratch s;
        if (!scratch_alloc(g, &s)) err = 1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nray; ++r) {
            if (err) { y[r] = 0.0; continue; }
            int iu = (int)(r % g->nu);
            int iv = (int)((r / g->nu) % g->nv);
            int a = (int)(r / ((int64_t)g->nu * g->nv));
            int n = trace_ray(g, a, iv, iu, &s);
            double acc = 0.0;
            for (int q = 0; q < n; ++q) acc += s.len[q] * x[s.idx[q]];
            y[r] = acc;
        }
        scratch_free(&s);
    }
    return err;
}

/*
 * x = A^T y by scattering the same segments.  Each thread accumulates into its
 * own volume over a static block of rays; the partial volumes are then summed
 * in thread order, so the result is deterministic for a given thread count.
 */
int ora_adjoint(const ora_geom *g, const double *y, double *x)
{
    int64_t nray = (int64_t)g->na * g->nv * g->nu;
    int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nth * (size_t)nvox, sizeof(double));
    if (!part) return 1;
    int err = 0;
#pragma omp parallel num_threads(nth) reduction(| : err)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = part + (size_t)tid * (size_t)nvox;
        ora_scratch s;
        if (!scratch_alloc(g, &s)) err = 1;
#pragma omp for schedule(static)
        for (int64_t r = 0; r < nray; ++r) {
            if (err) continue;
            double yr = y[r];
            if (yr == 0.0) continue;
            int iu = (int)(r % g->nu);
            int iv = (int)((r / g->nu) % g->nv);
            int a = (int)(r / ((int64_t)g->nu * g->nv));
            int n = trace_ray(g, a, iv, iu, &s);
            for (int q = 0; q < n; ++q) acc[s.idx[q]] += s.len[q] * yr;
        }
        scratch_free(&s);
    }
    if (!err) {
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < nvox; ++j) {
            double v = 0.0;
            for (int t = 0; t < nth; ++t) v += part[(size_t)t * (size_t)nvox + j];
            x[j] = v;
        }
    }
    free(part);
    return err;
}

/*
 * Segments of one ray, for tests: writes up to `cap` (voxel index, length)
 * pairs and returns the segment count (or -1 if `cap` is too small).
 */
int ora_ray_segments(const ora_geom *g, int a, int iv, int iu, int64_t *idx, double *len, int cap)
{
    ora_scratch s;
    if (!scratch_alloc(g, &s)) return -1;
    int n = trace_ray(g, a, iv, iu, &s);
    if (n > cap) { scratch_free(&s); return -1; }
    memcpy(idx, s.idx, (size_t)n * sizeof(int64_t));
    memcpy(len, s.len, (size_t)n * sizeof(double));
    scratch_free(&s);
    return n;
}

/* Forward projection of a subset of rays (flat ray ids), for sampled checks. */
int ora_forward_rays(const ora_geom *g, const double *x, const int64_t *rays, int64_t nr, double *y)
{
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        ora_scratch s;
        if (!scratch_alloc(g, &s)) err = 1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < nr; ++q) {
            if (err) { y[q] = 0.0; continue; }
            int64_t r = rays[q];
            int iu = (int)(r % g->nu);
            int iv = (int)((r / g->nu) % g->nv);
            int a = (int)(r / ((int64_t)g->nu * g->nv));
            int n = trace_ray(g, a, iv, iu, &s);
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += s.len[k] * x[s.idx[k]];
            y[q] = acc;
        }
        scratch_free(&s);
    }
    return err;
}

/* Number of nonzero entries of A (segments of positive length), summed over
 * every ray: the count the algorithmic-traffic model of a sparse matvec uses.
 * Also returns the number of rays with at least one segment. */
int ora_count_nnz(const ora_geom *g, int64_t *nnz, int64_t *hit_rays)
{
    int64_t nray = (int64_t)g->na * g->nv * g->nu;
    int64_t tot = 0, hits = 0;
    int err = 0;
#pragma omp parallel reduction(+ : tot, hits) reduction(| : err)
    {
        ora_scratch s;
        if (!scratch_alloc(g, &s)) err = 1;
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < nray; ++r) {
            if (err) continue;
            int iu = (int)(r % g->nu);
            int iv = (int)((r / g->nu) % g->nv);
            int a = (int)(r / ((int64_t)g->nu * g->nv));
            int n = trace_ray(g, a, iv, iu, &s);
            tot += n;
            hits += n > 0;
        }
        scratch_free(&s);
    }
    *nnz = tot;
    *hit_rays = hits;
    return err;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by later calls.  The forward does not depend on the count; the
 * adjoint's per-thread partial volumes, summed in thread order, make its result
 * change with the count at FP64 rounding level. */
void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
