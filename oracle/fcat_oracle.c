/*
 * FP64 CPU oracle for the polyenergetic cone-beam projector.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the test suite, the smoke check and the
 * CPU baseline leg of the benchmark load it; the product library never does.
 * It shares no code, header, table or helper with the HIP path.
 *
 * What it computes (fastCAT, O'Connell & Bazalova-Carter, arXiv 2011.04736):
 *
 *  - Sec. II.F (Raytracing): a projection is the line integral of the
 *    attenuation coefficient along the source-to-pixel ray.  Sec. II.C
 *    stores the phantom as integer material labels, so mu(E, x) is
 *    mu_{label(x)}(E) and the line integral at every energy is
 *    P_e = sum_m mu_{m,e} L_m with L_m the length of the ray inside material
 *    m.  L is computed with Siddon's exact algorithm (R. L. Siddon, "Fast
 *    calculation of the exact radiological path for a three-dimensional CT
 *    array", Med. Phys. 12(2), 1985): the parametric positions of all voxel
 *    planes crossed are merged into one sorted list; each pair of
 *    neighbours bounds one voxel, found from its midpoint.
 *  - Sec. II.F, Eq. 3: the detected intensity is the spectrum- and
 *    response-weighted sum over energies of the intensity profiles, the
 *    scatter having been added to the primary profiles before weighting.
 *  - Sec. II.G: the profiles are convolved with the optical spread function
 *    (Eq. 1) of each energy (here: each energy group) and summed.
 *
 * Every quantity is double precision; float inputs are converted exactly.
 * Parallelism is plain OpenMP over rays; there is no blocking, fusion or
 * reordering beyond the definitions above.
 *
 * Conventions (the paper states none; these are the readings the build uses):
 *   world z is the rotation axis, the isocentre is the origin;
 *   source s = (SID cos t, SID sin t, 0);
 *   detector centre c = -(SDD - SID)(cos t, sin t, 0);
 *   u axis = (-sin t, cos t, 0), v axis = (0, 0, 1);
 *   pixel (iv, iu) centre = c + ((iu - (Nu-1)/2) du + off_u) u
 *                             + ((iv - (Nv-1)/2) dv + off_v) v;
 *   t_a = 2 pi a / A unless explicit angles are given;
 *   voxel (ix, iy, iz) is the half-open box [x0 + ix dx, x0 + (ix+1) dx) x ...
 *   with x0 = cx - Nx dx / 2 (same for y, z);
 *   labels are stored labels[iz][iy][ix], x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double sid, sdd;
    int32_t nu, nv;
    double du, dv, off_u, off_v;
    int32_t n_angles;
    const double *angles; /* NULL: 2 pi a / A */
} orc_geometry;

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double cx, cy, cz;
    const int8_t *labels; /* [nz][ny][nx] */
} orc_volume;

enum { ORC_OK = 0, ORC_BAD_LABEL = 1, ORC_NOMEM = 2, ORC_BAD_ARG = 3 };

static void set_threads(int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------ geometry */

double orc_angle(const orc_geometry *g, int a)
{
    if (g->angles) return g->angles[a];
    return 2.0 * M_PI * (double)a / (double)g->n_angles;
}

/* Source point and pixel-centre point of ray (a, iv, iu). */
void orc_ray_endpoints(const orc_geometry *g, int a, int iv, int iu, double src[3], double dst[3])
{
    double t = orc_angle(g, a);
    double ct = cos(t), st = sin(t);
    double pu = ((double)iu - 0.5 * (double)(g->nu - 1)) * g->du + g->off_u;
    double pv = ((double)iv - 0.5 * (double)(g->nv - 1)) * g->dv + g->off_v;
    double back = g->sdd - g->sid;
    src[0] = g->sid * ct;
    src[1] = g->sid * st;
    src[2] = 0.0;
    dst[0] = -back * ct - pu * st;
    dst[1] = -back * st + pu * ct;
    dst[2] = pv;
}

/* ---------------------------------------------------- Siddon, merged alpha */

typedef struct {
    double lo[3];   /* first plane of each axis */
    double h[3];    /* voxel size per axis */
    int32_t n[3];   /* voxel count per axis */
} box_t;

static box_t make_box(const orc_volume *v)
{
    box_t b;
    b.n[0] = v->nx; b.n[1] = v->ny; b.n[2] = v->nz;
    b.h[0] = v->dx; b.h[1] = v->dy; b.h[2] = v->dz;
    b.lo[0] = v->cx - 0.5 * v->nx * v->dx;
    b.lo[1] = v->cy - 0.5 * v->ny * v->dy;
    b.lo[2] = v->cz - 0.5 * v->nz * v->dz;
    return b;
}

/* Parametric plane positions of one axis, increasing, strictly inside (amin, amax). */
static int axis_alphas(const box_t *b, int ax, const double s[3], const double d[3],
                       double amin, double amax, double *out)
{
    int cnt = 0;
    if (d[ax] == 0.0) return 0;
    int n = b->n[ax];
    if (d[ax] > 0.0) {
        for (int i = 0; i <= n; ++i) {
            double a = (b->lo[ax] + i * b->h[ax] - s[ax]) / d[ax];
            if (a > amin && a < amax) out[cnt++] = a;
        }
    } else {
        for (int i = n; i >= 0; --i) {
            double a = (b->lo[ax] + i * b->h[ax] - s[ax]) / d[ax];
            if (a > amin && a < amax) out[cnt++] = a;
        }
    }
    return cnt;
}

static int clampi(int i, int n)
{
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/*
 * Path length of segment src->dst inside each material.  `work` must hold
 * 2 * (nx + ny + nz + 5) doubles.  L[0..n_mat-1] is overwritten.
 */
static int siddon_work(const double src[3], const double dst[3], const orc_volume *v,
                       int n_mat, double *L, double *work)
{
    box_t b = make_box(v);
    double d[3] = {dst[0] - src[0], dst[1] - src[1], dst[2] - src[2]};
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int m = 0; m < n_mat; ++m) L[m] = 0.0;

    double amin = 0.0, amax = 1.0;
    for (int ax = 0; ax < 3; ++ax) {
        double lo = b.lo[ax], hi = b.lo[ax] + b.n[ax] * b.h[ax];
        if (d[ax] == 0.0) {
            if (!(src[ax] >= lo && src[ax] < hi)) return ORC_OK; /* parallel and outside */
            continue;
        }
        double a0 = (lo - src[ax]) / d[ax];
        double a1 = (hi - src[ax]) / d[ax];
        double amn = a0 < a1 ? a0 : a1, amx = a0 < a1 ? a1 : a0;
        if (amn > amin) amin = amn;
        if (amx < amax) amax = amx;
    }
    if (!(amax > amin)) return ORC_OK; /* misses the grid */

    int cap = b.n[0] + b.n[1] + b.n[2] + 5;
    double *lists = work;           /* three concatenated axis lists */
    double *merged = work + cap;
    int cnt[3], off[3], o = 0;
    for (int ax = 0; ax < 3; ++ax) {
        off[ax] = o;
        cnt[ax] = axis_alphas(&b, ax, src, d, amin, amax, lists + o);
        o += cnt[ax];
    }
    /* merge the three increasing lists between amin and amax */
    int k = 0, p[3] = {0, 0, 0};
    merged[k++] = amin;
    for (;;) {
        int best = -1;
        double bv = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            if (p[ax] < cnt[ax]) {
                double a = lists[off[ax] + p[ax]];
                if (best < 0 || a < bv) { best = ax; bv = a; }
            }
        }
        if (best < 0) break;
        merged[k++] = bv;
        p[best]++;
    }
    merged[k++] = amax;

    for (int i = 0; i + 1 < k; ++i) {
        double a0 = merged[i], a1 = merged[i + 1];
        if (!(a1 > a0)) continue; /* coincident planes: zero-length segment */
        double am = 0.5 * (a0 + a1);
        int ix = clampi((int)floor((src[0] + am * d[0] - b.lo[0]) / b.h[0]), b.n[0]);
        int iy = clampi((int)floor((src[1] + am * d[1] - b.lo[1]) / b.h[1]), b.n[1]);
        int iz = clampi((int)floor((src[2] + am * d[2] - b.lo[2]) / b.h[2]), b.n[2]);
        int lab = v->labels[((int64_t)iz * b.n[1] + iy) * b.n[0] + ix];
        if (lab < 0 || lab >= n_mat) return ORC_BAD_LABEL;
        L[lab] += (a1 - a0) * len;
    }
    return ORC_OK;
}

int orc_siddon(const double src[3], const double dst[3], const orc_volume *v, int n_mat, double *L)
{
    size_t cap = (size_t)(v->nx + v->ny + v->nz + 5);
    double *work = (double *)malloc(2 * cap * sizeof(double));
    if (!work) return ORC_NOMEM;
    int rc = siddon_work(src, dst, v, n_mat, L, work);
    free(work);
    return rc;
}

/*
 * Independent brute-force path lengths: midpoint rule with n_steps equal
 * steps over the whole segment src->dst, each step charged to the voxel
 * (half-open boxes) holding its midpoint, nothing outside the grid.
 * Error per material is at most one step length per label change.
 */
int orc_bruteforce(const double src[3], const double dst[3], const orc_volume *v, int n_mat,
                   int64_t n_steps, double *L)
{
    box_t b = make_box(v);
    double d[3] = {dst[0] - src[0], dst[1] - src[1], dst[2] - src[2]};
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double step = len / (double)n_steps;
    for (int m = 0; m < n_mat; ++m) L[m] = 0.0;
    for (int64_t k = 0; k < n_steps; ++k) {
        double a = ((double)k + 0.5) / (double)n_steps;
        int idx[3];
        int inside = 1;
        for (int ax = 0; ax < 3; ++ax) {
            double q = floor((src[ax] + a * d[ax] - b.lo[ax]) / b.h[ax]);
            if (q < 0.0 || q >= (double)b.n[ax]) { inside = 0; break; }
            idx[ax] = (int)q;
        }
        if (!inside) continue;
        int lab = v->labels[((int64_t)idx[2] * b.n[1] + idx[1]) * b.n[0] + idx[0]];
        if (lab < 0 || lab >= n_mat) return ORC_BAD_LABEL;
        L[lab] += step;
    }
    return ORC_OK;
}

/*
 * Path lengths of a list of rays.  ray_id = (a * nv + iv) * nu + iu.
 * L is [n][n_mat].
 */
int orc_pathlengths_rays(const orc_geometry *g, const orc_volume *v, int n_mat,
                         const int64_t *ray_ids, int64_t n, double *L, int n_threads)
{
    set_threads(n_threads);
    int rc = ORC_OK;
    size_t cap = (size_t)(v->nx + v->ny + v->nz + 5);
#pragma omp parallel
    {
        double *work = (double *)malloc(2 * cap * sizeof(double));
        int local = work ? ORC_OK : ORC_NOMEM;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n; ++r) {
            if (local != ORC_OK) continue;
            int64_t id = ray_ids[r];
            int iu = (int)(id % g->nu);
            int iv = (int)((id / g->nu) % g->nv);
            int a = (int)(id / ((int64_t)g->nu * g->nv));
            double s[3], p[3];
            orc_ray_endpoints(g, a, iv, iu, s, p);
            int e = siddon_work(s, p, v, n_mat, L + r * n_mat, work);
            if (e != ORC_OK) local = e;
        }
        if (local != ORC_OK) {
#pragma omp critical
            rc = local;
        }
        free(work);
    }
    return rc;
}

/* Path lengths of every pixel of the listed angles: L is [n_ang][nv][nu][n_mat]. */
int orc_pathlengths(const orc_geometry *g, const orc_volume *v, int n_mat,
                    const int32_t *angle_idx, int n_ang, double *L, int n_threads)
{
    int64_t per = (int64_t)g->nu * g->nv;
    int64_t n = per * n_ang;
    int64_t *ids = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!ids) return ORC_NOMEM;
    for (int k = 0; k < n_ang; ++k)
        for (int64_t p = 0; p < per; ++p) ids[k * per + p] = (int64_t)angle_idx[k] * per + p;
    int rc = orc_pathlengths_rays(g, v, n_mat, ids, n, L, n_threads);
    free(ids);
    return rc;
}

/* ------------------------------------------------------ spectral (Eq. 3) */

/*
 * Y[g][r] = sum_{e : group[e] == g} phi_e eta_e (I0_r exp(-P_{r,e}) + s_e S_r),
 * P_{r,e} = sum_m mu[m][e] L[r][m].  i0 NULL means 1, S NULL means 0,
 * s_bin NULL means 1.  Sums run in bin order.
 */
void orc_spectral(const double *L, int64_t n, int n_mat, int n_energy, int n_groups,
                  const double *mu, const double *phi, const double *eta, const int32_t *group,
                  const double *i0, const double *S, const double *s_bin, double *Y, int n_threads)
{
    set_threads(n_threads);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        for (int gi = 0; gi < n_groups; ++gi) Y[(int64_t)gi * n + r] = 0.0;
        double flood = i0 ? i0[r] : 1.0;
        double sc = S ? S[r] : 0.0;
        for (int e = 0; e < n_energy; ++e) {
            double P = 0.0;
            for (int m = 0; m < n_mat; ++m) P += mu[(int64_t)m * n_energy + e] * L[r * n_mat + m];
            double w = phi[e] * eta[e];
            double se = s_bin ? s_bin[e] : 1.0;
            Y[(int64_t)group[e] * n + r] += w * (flood * exp(-P) + se * sc);
        }
    }
}

/* ------------------------------------------------- optical spread (Sec. II.G) */

/*
 * out[a][v][u] = sum_g sum_{p,q} K[g][p][q] Y[a][g][v - p + c][u - q + c],
 * c = (k-1)/2, zero outside the detector (same-size true convolution).
 */
void orc_psf(const double *Y, int n_ang, int n_groups, int nv, int nu, const double *K, int k,
             double *out, int n_threads)
{
    set_threads(n_threads);
    int c = (k - 1) / 2;
    int64_t plane = (int64_t)nv * nu;
#pragma omp parallel for collapse(2) schedule(static)
    for (int a = 0; a < n_ang; ++a) {
        for (int v = 0; v < nv; ++v) {
            for (int u = 0; u < nu; ++u) {
                double acc = 0.0;
                for (int gi = 0; gi < n_groups; ++gi) {
                    const double *Yg = Y + ((int64_t)a * n_groups + gi) * plane;
                    const double *Kg = K + (int64_t)gi * k * k;
                    for (int p = 0; p < k; ++p) {
                        int vv = v - p + c;
                        if (vv < 0 || vv >= nv) continue;
                        for (int q = 0; q < k; ++q) {
                            int uu = u - q + c;
                            if (uu < 0 || uu >= nu) continue;
                            acc += Kg[p * k + q] * Yg[(int64_t)vv * nu + uu];
                        }
                    }
                }
                out[(int64_t)a * plane + (int64_t)v * nu + u] = acc;
            }
        }
    }
}

/* ------------------------------------------------------ whole projector */

/*
 * Projections of the listed angles.
 *   S      [n_ang][nv][nu] scatter maps of those angles, or NULL (off);
 *   flood  [nv][nu] or NULL (= 1);
 *   K      [G][k][k] or NULL (off: out = sum_g Y_g);
 *   out    [n_ang][nv][nu];
 *   Y_out  [n_ang][G][nv][nu] group signals before the spread, or NULL.
 */
int orc_project(const orc_geometry *g, const orc_volume *v, int n_mat, int n_energy, int n_groups,
                const double *mu, const double *phi, const double *eta, const int32_t *group,
                const double *flood, const double *S, const double *s_bin,
                const double *K, int k, const int32_t *angle_idx, int n_ang,
                double *out, double *Y_out, int n_threads)
{
    int64_t plane = (int64_t)g->nu * g->nv;
    int64_t n = plane * n_ang;
    double *L = (double *)malloc((size_t)n * n_mat * sizeof(double));
    double *Yr = (double *)malloc((size_t)n * n_groups * sizeof(double));
    double *i0 = flood ? (double *)malloc((size_t)n * sizeof(double)) : NULL;
    double *Y = Y_out ? Y_out : (double *)malloc((size_t)n * n_groups * sizeof(double));
    if (!L || !Yr || (flood && !i0) || !Y) {
        free(L); free(Yr); free(i0);
        if (!Y_out) free(Y);
        return ORC_NOMEM;
    }
    int rc = orc_pathlengths(g, v, n_mat, angle_idx, n_ang, L, n_threads);
    if (rc == ORC_OK) {
        if (flood)
            for (int a = 0; a < n_ang; ++a) memcpy(i0 + a * plane, flood, (size_t)plane * sizeof(double));
        /* Yr is [G][n] with n = all rays of all listed angles */
        orc_spectral(L, n, n_mat, n_energy, n_groups, mu, phi, eta, group, i0, S, s_bin, Yr, n_threads);
        for (int a = 0; a < n_ang; ++a)
            for (int gi = 0; gi < n_groups; ++gi)
                memcpy(Y + ((int64_t)a * n_groups + gi) * plane, Yr + (int64_t)gi * n + a * plane,
                       (size_t)plane * sizeof(double));
        if (K) {
            orc_psf(Y, n_ang, n_groups, g->nv, g->nu, K, k, out, n_threads);
        } else {
            for (int a = 0; a < n_ang; ++a)
                for (int64_t p = 0; p < plane; ++p) {
                    double acc = 0.0;
                    for (int gi = 0; gi < n_groups; ++gi) acc += Y[((int64_t)a * n_groups + gi) * plane + p];
                    out[a * plane + p] = acc;
                }
        }
    }
    free(L); free(Yr); free(i0);
    if (!Y_out) free(Y);
    return rc;
}

/* ------------------------------------------ projector of a voxel image, Aᵀ */
/*
 * The projector of a real-valued voxel image f (the line integral of Sec.
 * II.F over an image instead of a labelled phantom, as an iterative
 * reconstruction uses it, Sec. II.G) and its transpose:
 *   (A f)_r     = sum over the voxels k the ray r crosses of l_{r,k} f_k,
 *   (A^T y)_k   = sum over the rays r of l_{r,k} y_r,
 * with l_{r,k} the length of ray r inside voxel k from Siddon's merged
 * parametric plane crossings (as siddon_work above).  The grid follows the
 * phantom's conventions; f and the result of A^T are [nz][ny][nx].
 */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double cx, cy, cz;
} orc_grid;

typedef void (*orc_visit_fn)(void *ctx, int64_t voxel, double length);

/* Calls visit(ctx, voxel, length) for each voxel segment of src->dst, in order. */
static void siddon_visit(const double src[3], const double dst[3], const orc_grid *gr, double *work,
                         orc_visit_fn visit, void *ctx)
{
    box_t b;
    b.n[0] = gr->nx; b.n[1] = gr->ny; b.n[2] = gr->nz;
    b.h[0] = gr->dx; b.h[1] = gr->dy; b.h[2] = gr->dz;
    b.lo[0] = gr->cx - 0.5 * gr->nx * gr->dx;
    b.lo[1] = gr->cy - 0.5 * gr->ny * gr->dy;
    b.lo[2] = gr->cz - 0.5 * gr->nz * gr->dz;
    double d[3] = {dst[0] - src[0], dst[1] - src[1], dst[2] - src[2]};
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double amin = 0.0, amax = 1.0;
    for (int ax = 0; ax < 3; ++ax) {
        double lo = b.lo[ax], hi = b.lo[ax] + b.n[ax] * b.h[ax];
        if (d[ax] == 0.0) {
            if (!(src[ax] >= lo && src[ax] < hi)) return;
            continue;
        }
        double a0 = (lo - src[ax]) / d[ax], a1 = (hi - src[ax]) / d[ax];
        double amn = a0 < a1 ? a0 : a1, amx = a0 < a1 ? a1 : a0;
        if (amn > amin) amin = amn;
        if (amx < amax) amax = amx;
    }
    if (!(amax > amin)) return;
    int cap = b.n[0] + b.n[1] + b.n[2] + 5;
    double *lists = work, *merged = work + cap;
    int cnt[3], off[3], o = 0;
    for (int ax = 0; ax < 3; ++ax) {
        off[ax] = o;
        cnt[ax] = axis_alphas(&b, ax, src, d, amin, amax, lists + o);
        o += cnt[ax];
    }
    int k = 0, p[3] = {0, 0, 0};
    merged[k++] = amin;
    for (;;) {
        int best = -1;
        double bv = 0.0;
        for (int ax = 0; ax < 3; ++ax)
            if (p[ax] < cnt[ax]) {
                double a = lists[off[ax] + p[ax]];
                if (best < 0 || a < bv) { best = ax; bv = a; }
            }
        if (best < 0) break;
        merged[k++] = bv;
        p[best]++;
    }
    merged[k++] = amax;
    for (int i = 0; i + 1 < k; ++i) {
        double a0 = merged[i], a1 = merged[i + 1];
        if (!(a1 > a0)) continue;
        double am = 0.5 * (a0 + a1);
        int ix = clampi((int)floor((src[0] + am * d[0] - b.lo[0]) / b.h[0]), b.n[0]);
        int iy = clampi((int)floor((src[1] + am * d[1] - b.lo[1]) / b.h[1]), b.n[1]);
        int iz = clampi((int)floor((src[2] + am * d[2] - b.lo[2]) / b.h[2]), b.n[2]);
        visit(ctx, ((int64_t)iz * b.n[1] + iy) * b.n[0] + ix, (a1 - a0) * len);
    }
}

typedef struct { const double *f; double sum; } fwd_ctx;
static void fwd_visit(void *c, int64_t voxel, double length)
{
    fwd_ctx *x = (fwd_ctx *)c;
    x->sum += length * x->f[voxel];
}

typedef struct { double *img; double y; } bp_ctx;
static void bp_visit(void *c, int64_t voxel, double length)
{
    bp_ctx *x = (bp_ctx *)c;
    double v = x->y * length;
#pragma omp atomic
    x->img[voxel] += v;
}

/* proj[n_ang][nv][nu] = (A f) over every pixel of the listed angles. */
int orc_forward_image(const orc_geometry *g, const orc_grid *gr, const double *f, const int32_t *angle_idx,
                      int n_ang, double *proj, int n_threads)
{
    set_threads(n_threads);
    int rc = ORC_OK;
    size_t cap = (size_t)(gr->nx + gr->ny + gr->nz + 5);
    int64_t plane = (int64_t)g->nu * g->nv, n = (int64_t)n_ang * plane;
#pragma omp parallel
    {
        double *work = (double *)malloc(2 * cap * sizeof(double));
        if (!work) {
#pragma omp critical
            rc = ORC_NOMEM;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n; ++r) {
            if (!work) continue;
            int a = angle_idx[r / plane];
            int iv = (int)((r % plane) / g->nu), iu = (int)(r % g->nu);
            double s[3], p[3];
            orc_ray_endpoints(g, a, iv, iu, s, p);
            fwd_ctx c = {f, 0.0};
            siddon_visit(s, p, gr, work, fwd_visit, &c);
            proj[r] = c.sum;
        }
        free(work);
    }
    return rc;
}

/* img[nz][ny][nx] += (A^T y) over every pixel of the listed angles (y [n_ang][nv][nu]). */
int orc_backproject_image(const orc_geometry *g, const orc_grid *gr, const double *y, const int32_t *angle_idx,
                          int n_ang, double *img, int n_threads)
{
    set_threads(n_threads);
    int rc = ORC_OK;
    size_t cap = (size_t)(gr->nx + gr->ny + gr->nz + 5);
    int64_t plane = (int64_t)g->nu * g->nv, n = (int64_t)n_ang * plane;
#pragma omp parallel
    {
        double *work = (double *)malloc(2 * cap * sizeof(double));
        if (!work) {
#pragma omp critical
            rc = ORC_NOMEM;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n; ++r) {
            if (!work || y[r] == 0.0) continue;
            int a = angle_idx[r / plane];
            int iv = (int)((r % plane) / g->nu), iu = (int)(r % g->nu);
            double s[3], p[3];
            orc_ray_endpoints(g, a, iv, iu, s, p);
            bp_ctx c = {img, y[r]};
            siddon_visit(s, p, gr, work, bp_visit, &c);
        }
        free(work);
    }
    return rc;
}
