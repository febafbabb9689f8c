// C ABI of libfcat.so: host-side argument validation, workspace layout,
// angle chunking and kernel launches.  See include/fcat.h for the contract.
#include "fcat_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace fcat {
namespace {

thread_local std::string g_last_error;

fcat_status fail(fcat_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

fcat_status device_fail(hipError_t e, const char *where)
{
    return fail(FCAT_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

fcat_status check_geometry(const fcat_geometry_t *g)
{
    if (!g) return fail(FCAT_E_INVALID_ARG, "geometry is NULL");
    if (!finite_pos(g->sid_mm)) return fail(FCAT_E_INVALID_ARG, "sid_mm must be finite and > 0");
    if (!std::isfinite(g->sdd_mm) || !(g->sdd_mm > g->sid_mm))
        return fail(FCAT_E_INVALID_ARG, "sdd_mm must be finite and > sid_mm");
    if (g->nu < 1 || g->nv < 1 || g->n_angles < 1)
        return fail(FCAT_E_INVALID_ARG, "nu, nv and n_angles must be >= 1");
    if ((int64_t)g->nu * g->nv > (int64_t)1 << 30)
        return fail(FCAT_E_INVALID_ARG, "detector larger than 2^30 pixels");
    if (!finite_pos(g->du_mm) || !finite_pos(g->dv_mm))
        return fail(FCAT_E_INVALID_ARG, "du_mm and dv_mm must be finite and > 0");
    if (!std::isfinite(g->off_u_mm) || !std::isfinite(g->off_v_mm))
        return fail(FCAT_E_INVALID_ARG, "detector offsets must be finite");
    return FCAT_OK;
}

fcat_status check_phantom(const fcat_phantom_t *p)
{
    if (!p) return fail(FCAT_E_INVALID_ARG, "phantom is NULL");
    if (!p->labels) return fail(FCAT_E_INVALID_ARG, "phantom labels is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(FCAT_E_INVALID_ARG, "nx, ny, nz must be >= 1");
    if ((int64_t)p->nx * p->ny * p->nz >= ((int64_t)1 << 31))
        return fail(FCAT_E_INVALID_ARG, "phantom larger than 2^31 - 1 voxels");
    if (!finite_pos(p->dx_mm) || !finite_pos(p->dy_mm) || !finite_pos(p->dz_mm))
        return fail(FCAT_E_INVALID_ARG, "voxel sizes must be finite and > 0");
    if (!std::isfinite(p->cx_mm) || !std::isfinite(p->cy_mm) || !std::isfinite(p->cz_mm))
        return fail(FCAT_E_INVALID_ARG, "grid centre must be finite");
    return FCAT_OK;
}

int padded_materials(int m) { return m <= 8 ? 8 : (m <= 16 ? 16 : 32); }

// Validates the spectral descriptor and fills the host part of the tables.
fcat_status check_spectral(const fcat_spectral_t *s, bool need_tables, SpecTables &t)
{
    if (!s) return fail(FCAT_E_INVALID_ARG, "spectral is NULL");
    if (s->n_mat < 1 || s->n_mat > FCAT_MAX_MATERIALS)
        return fail(FCAT_E_INVALID_ARG, "n_mat must be in 1..%d", FCAT_MAX_MATERIALS);
    if (s->n_energy < 1 || s->n_energy > FCAT_MAX_ENERGIES)
        return fail(FCAT_E_INVALID_ARG, "n_energy must be in 1..%d", FCAT_MAX_ENERGIES);
    if (s->n_groups < 1 || s->n_groups > FCAT_MAX_GROUPS || s->n_groups > s->n_energy)
        return fail(FCAT_E_INVALID_ARG, "n_groups must be in 1..min(n_energy, %d)", FCAT_MAX_GROUPS);
    if (need_tables && (!s->mu || !s->phi || !s->eta))
        return fail(FCAT_E_INVALID_ARG, "mu, phi and eta must not be NULL");
    t.E = s->n_energy;
    t.M = s->n_mat;
    t.G = s->n_groups;
    t.mp = padded_materials(s->n_mat);
    for (int g = 0; g <= FCAT_MAX_GROUPS; ++g) t.gstart[g] = t.E;
    if (!s->group_of_bin) {
        for (int g = 0; g < t.G; ++g) {
            // first e with floor(e G / E) == g
            t.gstart[g] = (int)(((int64_t)g * t.E + t.G - 1) / t.G);
        }
    } else {
        int prev = -1;
        for (int e = 0; e < t.E; ++e) {
            const int g = s->group_of_bin[e];
            if (g < 0 || g >= t.G) return fail(FCAT_E_INVALID_ARG, "group_of_bin[%d] = %d not in [0, %d)", e, g, t.G);
            if (g < prev) return fail(FCAT_E_INVALID_ARG, "group_of_bin must be non-decreasing (bin %d)", e);
            if (g > prev + 1) return fail(FCAT_E_INVALID_ARG, "group %d has no energy bin", prev + 1);
            if (g != prev) t.gstart[g] = e;
            prev = g;
        }
        if (prev != t.G - 1) return fail(FCAT_E_INVALID_ARG, "group %d has no energy bin", prev + 1);
    }
    t.gstart[t.G] = t.E;
    return FCAT_OK;
}

fcat_status check_psf(const fcat_psf_t *p)
{
    if (!p) return FCAT_OK;
    if (!p->kernels) return fail(FCAT_E_INVALID_ARG, "psf kernels is NULL");
    if (p->k < 1 || p->k > FCAT_MAX_PSF || (p->k % 2) == 0)
        return fail(FCAT_E_INVALID_ARG, "psf k must be odd and in 1..%d", FCAT_MAX_PSF);
    return FCAT_OK;
}

size_t brick_count(const fcat_phantom_t *p)
{
    return (size_t)((p->nx + kBrickEdge - 1) / kBrickEdge) * ((p->ny + kBrickEdge - 1) / kBrickEdge) *
           ((p->nz + kBrickEdge - 1) / kBrickEdge);
}

// brick map + brick-major label copy
size_t brick_bytes(const fcat_phantom_t *p) { return align_up(brick_count(p)) + brick_count(p) * kBrickVox; }

TraceGeom make_geom(const fcat_geometry_t *g, const fcat_phantom_t *p)
{
    TraceGeom G{};
    G.sid = g->sid_mm;
    G.back = g->sdd_mm - g->sid_mm;
    G.du = g->du_mm;
    G.dv = g->dv_mm;
    G.off_u = g->off_u_mm;
    G.off_v = g->off_v_mm;
    G.cu = 0.5 * (g->nu - 1);
    G.cv = 0.5 * (g->nv - 1);
    const double h[3] = {p->dx_mm, p->dy_mm, p->dz_mm};
    const double c[3] = {p->cx_mm, p->cy_mm, p->cz_mm};
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int ax = 0; ax < 3; ++ax) {
        G.h[ax] = h[ax];
        G.inv_h[ax] = 1.0 / h[ax];
        G.n[ax] = n[ax];
        G.lo[ax] = c[ax] - 0.5 * n[ax] * h[ax];
    }
    G.nu = g->nu;
    G.nv = g->nv;
    G.n_angles = g->n_angles;
    G.angles = g->angles_rad;
    for (int ax = 0; ax < 3; ++ax) G.nb[ax] = (n[ax] + kBrickEdge - 1) / kBrickEdge;
    G.bricks = nullptr;
    G.labels_bm = nullptr;
    return G;
}

struct Layout {
    size_t flags, muT, w, Wg, Wsg, afrag, wtile, bricks, Y, fixed;
    size_t per_angle;  // bytes of group signal per angle (0 without psf)
};

// Host part of the split-precision tables: group-aligned tiles of 16 bins.
void split_host(const SpecTables &t, SplitTables &sp)
{
    int T = 0;
    for (int g = 0; g < t.G; ++g) {
        sp.gtile[g] = T;
        T += (t.gstart[g + 1] - t.gstart[g] + 15) / 16;
    }
    for (int g = t.G; g <= FCAT_MAX_GROUPS; ++g) sp.gtile[g] = T;
    sp.T = T;
    sp.nkb = (3 * t.M + 31) / 32;
}

Layout layout(const SpecTables &t, const fcat_geometry_t *g, bool with_psf, size_t nbricks = 0,
              const SplitTables *sp = nullptr)
{
    Layout L{};
    size_t o = 0;
    L.flags = o;
    o += align_up(64 * sizeof(int));
    L.muT = o;
    o += align_up((size_t)t.E * t.mp * sizeof(float));
    L.w = o;
    o += align_up((size_t)t.E * sizeof(float));
    L.Wg = o;
    o += align_up((size_t)t.G * sizeof(float));
    L.Wsg = o;
    o += align_up((size_t)t.G * sizeof(float));
    L.afrag = o;
    if (sp) o += align_up((size_t)sp->T * sp->nkb * kWave * 16);
    L.wtile = o;
    if (sp) o += align_up((size_t)sp->T * 16 * sizeof(float));
    L.bricks = o;
    o += align_up(nbricks);
    L.Y = o;
    L.fixed = o;
    L.per_angle = (with_psf && g) ? align_up((size_t)t.G * g->nu * g->nv * sizeof(float)) : 0;
    return L;
}

constexpr size_t kDefaultChunkBytes = (size_t)1 << 30;

int default_chunk(const Layout &L, int n_angles)
{
    if (L.per_angle == 0) return n_angles;
    size_t c = kDefaultChunkBytes / L.per_angle;
    if (c < 1) c = 1;
    if (c > (size_t)n_angles) c = (size_t)n_angles;
    return (int)c;
}

fcat_status check_workspace(void *ws, size_t have, size_t need)
{
    if (need == 0) return FCAT_OK;
    if (!ws) return fail(FCAT_E_WORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if ((uintptr_t)ws % kAlign) return fail(FCAT_E_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    if (have < need) return fail(FCAT_E_WORKSPACE, "workspace has %zu bytes, %zu needed", have, need);
    return FCAT_OK;
}

// ------------------------------------------------------------ kernel timing

std::mutex g_tmu;
bool g_timing = false;
struct Timed {
    int stage;
    hipEvent_t a, b;
};
std::vector<Timed> g_timed;
std::vector<hipEvent_t> g_free_events;

hipEvent_t take_event()
{
    if (!g_free_events.empty()) {
        hipEvent_t e = g_free_events.back();
        g_free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when timing is on.
struct StageTimer {
    int idx = -1;
    hipStream_t stream;
    StageTimer(int stage, hipStream_t s) : stream(s)
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        if (!g_timing) return;
        Timed t{stage, take_event(), take_event()};
        if (!t.a || !t.b) return;
        (void)hipEventRecord(t.a, s);
        g_timed.push_back(t);
        idx = (int)g_timed.size() - 1;
    }
    ~StageTimer()
    {
        if (idx < 0) return;
        std::lock_guard<std::mutex> lk(g_tmu);
        (void)hipEventRecord(g_timed[idx].b, stream);
    }
};

template <typename T>
T *at(void *base, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(base) + off); }

fcat_status prep_tables(const fcat_spectral_t *s, const float *s_bin, SpecTables &t, const Layout &L,
                        void *ws, hipStream_t stream)
{
    float *muT = at<float>(ws, L.muT), *w = at<float>(ws, L.w);
    float *Wg = at<float>(ws, L.Wg), *Wsg = at<float>(ws, L.Wsg);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        e = launch_prep_tables(s->mu, s->phi, s->eta, s_bin, t, muT, w, Wg, Wsg, stream);
    }
    if (e != hipSuccess) return device_fail(e, "prep_tables");
    t.muT = muT;
    t.w = w;
    t.Wg = Wg;
    t.Wsg = Wsg;
    return FCAT_OK;
}


fcat_status prep_split(const fcat_spectral_t *s, const SpecTables &t, SplitTables &sp, const Layout &L, void *ws,
                       hipStream_t stream)
{
    uint4 *afrag = at<uint4>(ws, L.afrag);
    float *wtile = at<float>(ws, L.wtile);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        e = launch_prep_split(s->mu, t, sp, afrag, wtile, stream);
    }
    if (e != hipSuccess) return device_fail(e, "prep_split");
    sp.afrag = afrag;
    sp.wtile = wtile;
    return FCAT_OK;
}

fcat_status check_pending()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return device_fail(e, "pending HIP error");
    return FCAT_OK;
}

}  // namespace
}  // namespace fcat

using namespace fcat;

extern "C" {

const char *fcat_status_string(fcat_status s)
{
    switch (s) {
    case FCAT_OK: return "ok";
    case FCAT_E_INVALID_ARG: return "invalid argument";
    case FCAT_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case FCAT_E_LABEL_RANGE: return "phantom label outside 0..n_mat-1";
    case FCAT_E_NONFINITE: return "non-finite value in an input table";
    case FCAT_E_DEVICE: return "HIP runtime error";
    case FCAT_E_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char *fcat_last_error(void) { return g_last_error.c_str(); }

int fcat_version(void) { return FCAT_VERSION; }

size_t fcat_project_workspace_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                    const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                                    const fcat_psf_t *psf, fcat_mode mode, int32_t angles_per_chunk)
{
    (void)scatter;
    SpecTables t{};
    if (check_geometry(geometry) || check_phantom(phantom) || check_spectral(spectral, false, t) ||
        check_psf(psf))
        return 0;
    SplitTables sp{};
    split_host(t, sp);
    Layout L = layout(t, geometry, psf != nullptr, brick_bytes(phantom), mode == FCAT_MODE_SPLIT_BF16 ? &sp : nullptr);
    int chunk = angles_per_chunk > 0 ? angles_per_chunk : default_chunk(L, geometry->n_angles);
    if (chunk > geometry->n_angles) chunk = geometry->n_angles;
    return L.fixed + (size_t)chunk * L.per_angle;
}

fcat_status fcat_project(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                         const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                         const fcat_psf_t *psf, fcat_mode mode, const fcat_surrogate_t *surrogate,
                         float *out, void *workspace, size_t workspace_bytes, void *stream_)
{
    (void)surrogate;
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_geometry(geometry)) || (s = check_phantom(phantom)) ||
        (s = check_spectral(spectral, true, t)) || (s = check_psf(psf)))
        return s;
    if (!out) return fail(FCAT_E_INVALID_ARG, "out is NULL");
    if (scatter && !scatter->maps) return fail(FCAT_E_INVALID_ARG, "scatter maps is NULL");
    if (mode != FCAT_MODE_PLAIN && mode != FCAT_MODE_SPLIT_BF16 && mode != FCAT_MODE_SURROGATE)
        return fail(FCAT_E_INVALID_ARG, "unknown mode %d", (int)mode);
    if (mode == FCAT_MODE_SURROGATE) return fail(FCAT_E_UNSUPPORTED, "surrogate mode is not built yet");
    const bool split = mode == FCAT_MODE_SPLIT_BF16;
    SplitTables sp{};
    split_host(t, sp);
    Layout L = layout(t, geometry, psf != nullptr, brick_bytes(phantom), split ? &sp : nullptr);
    const size_t need = L.fixed + L.per_angle;  // at least one angle per chunk
    if ((s = check_workspace(workspace, workspace_bytes, need))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);

    if ((s = prep_tables(spectral, scatter ? scatter->s_bin : nullptr, t, L, workspace, stream))) return s;
    if (split && (s = prep_split(spectral, t, sp, L, workspace, stream))) return s;
    TraceGeom G = make_geom(geometry, phantom);
    G.bricks = at<int8_t>(workspace, L.bricks);
    G.labels_bm = G.bricks + align_up(brick_count(phantom));
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        hipError_t e0 = launch_build_bricks(phantom->labels, phantom->nx, phantom->ny, phantom->nz,
                                            const_cast<int8_t *>(G.bricks), const_cast<int8_t *>(G.labels_bm),
                                            stream);
        if (e0 != hipSuccess) return device_fail(e0, "build_bricks");
    }
    const float *S = scatter ? scatter->maps : nullptr;
    const int A = geometry->n_angles;
    const int64_t plane = (int64_t)geometry->nu * geometry->nv;
    hipError_t e;
    auto rows = [&](int a0, int n, float *Yc, float *outc) {
        return split ? launch_project_rows_split(G, phantom->labels, t, sp, spectral->flood, S, a0, n, Yc, outc, stream)
                     : launch_project_rows(G, phantom->labels, t, spectral->flood, S, a0, n, Yc, outc, stream);
    };
    if (!psf) {
        StageTimer tm(FCAT_STAGE_TRACE, stream);
        e = rows(0, A, nullptr, out);
        if (e != hipSuccess) return device_fail(e, "project_rows");
        return FCAT_OK;
    }
    const int chunk = (int)std::min<size_t>((size_t)A, (workspace_bytes - L.fixed) / L.per_angle);
    float *Y = at<float>(workspace, L.Y);
    for (int a0 = 0; a0 < A; a0 += chunk) {
        const int n = std::min(chunk, A - a0);
        {
            StageTimer tm(FCAT_STAGE_TRACE, stream);
            e = rows(a0, n, Y, nullptr);
        }
        if (e != hipSuccess) return device_fail(e, "project_rows");
        {
            StageTimer tm(FCAT_STAGE_PSF, stream);
            e = launch_psf(Y, n, t.G, geometry->nv, geometry->nu, psf->kernels, psf->k, out + a0 * plane,
                           stream);
        }
        if (e != hipSuccess) return device_fail(e, "psf");
    }
    return FCAT_OK;
}

size_t fcat_pathlengths_workspace_bytes(const fcat_phantom_t *phantom)
{
    if (check_phantom(phantom)) return 0;
    return align_up(brick_bytes(phantom));
}

fcat_status fcat_pathlengths(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom, int32_t n_mat,
                             int32_t a_begin, int32_t a_end, float *L, void *workspace, size_t workspace_bytes,
                             void *stream_)
{
    g_last_error.clear();
    fcat_status s;
    if ((s = check_geometry(geometry)) || (s = check_phantom(phantom))) return s;
    if (n_mat < 1 || n_mat > FCAT_MAX_MATERIALS)
        return fail(FCAT_E_INVALID_ARG, "n_mat must be in 1..%d", FCAT_MAX_MATERIALS);
    if (a_begin < 0 || a_end > geometry->n_angles || a_begin >= a_end)
        return fail(FCAT_E_INVALID_ARG, "need 0 <= a_begin < a_end <= n_angles");
    if (!L) return fail(FCAT_E_INVALID_ARG, "L is NULL");
    if ((s = check_workspace(workspace, workspace_bytes, align_up(brick_bytes(phantom))))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    TraceGeom G = make_geom(geometry, phantom);
    int8_t *bricks = static_cast<int8_t *>(workspace);
    int8_t *labels_bm = bricks + align_up(brick_count(phantom));
    G.bricks = bricks;
    G.labels_bm = labels_bm;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        e = launch_build_bricks(phantom->labels, phantom->nx, phantom->ny, phantom->nz, bricks, labels_bm, stream);
    }
    if (e != hipSuccess) return device_fail(e, "build_bricks");
    {
        StageTimer tm(FCAT_STAGE_TRACE, stream);
        e = launch_pathlengths(G, phantom->labels, n_mat, a_begin, a_end - a_begin, L, stream);
    }
    if (e != hipSuccess) return device_fail(e, "pathlengths");
    return FCAT_OK;
}

size_t fcat_spectral_workspace_bytes(const fcat_spectral_t *spectral)
{
    SpecTables t{};
    if (check_spectral(spectral, false, t)) return 0;
    SplitTables sp{};
    split_host(t, sp);
    return layout(t, nullptr, false, 0, &sp).fixed;   // enough for either mode
}

fcat_status fcat_spectral(const float *Lin, int64_t n, const fcat_spectral_t *spectral, const float *i0,
                          const float *S, const float *s_bin, fcat_mode mode, float *Y, void *workspace,
                          size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_spectral(spectral, true, t))) return s;
    if (n < 0) return fail(FCAT_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!Lin || !Y)) return fail(FCAT_E_INVALID_ARG, "L and Y must not be NULL");
    if (mode != FCAT_MODE_PLAIN && mode != FCAT_MODE_SPLIT_BF16)
        return fail(FCAT_E_INVALID_ARG, "fcat_spectral takes PLAIN or SPLIT_BF16");
    const bool split = mode == FCAT_MODE_SPLIT_BF16;
    SplitTables sp{};
    split_host(t, sp);
    Layout L = layout(t, nullptr, false, 0, split ? &sp : nullptr);
    if ((s = check_workspace(workspace, workspace_bytes, L.fixed))) return s;
    if (n == 0) return FCAT_OK;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((s = prep_tables(spectral, s_bin, t, L, workspace, stream))) return s;
    if (split && (s = prep_split(spectral, t, sp, L, workspace, stream))) return s;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_TRACE, stream);
        e = split ? launch_spectral_split(Lin, n, t, sp, i0, S, Y, stream) : launch_spectral(Lin, n, t, i0, S, Y, stream);
    }
    if (e != hipSuccess) return device_fail(e, "spectral");
    return FCAT_OK;
}

fcat_status fcat_psf(const float *Y, int32_t n_ang, int32_t n_groups, int32_t nv, int32_t nu,
                     const fcat_psf_t *psf, float *out, void *stream)
{
    g_last_error.clear();
    fcat_status s;
    if (!psf) return fail(FCAT_E_INVALID_ARG, "psf is NULL");
    if ((s = check_psf(psf))) return s;
    if (n_ang < 1 || n_groups < 1 || n_groups > FCAT_MAX_GROUPS || nv < 1 || nu < 1)
        return fail(FCAT_E_INVALID_ARG, "sizes must be >= 1 (n_groups <= %d)", FCAT_MAX_GROUPS);
    if (n_ang > 65535) return fail(FCAT_E_INVALID_ARG, "n_ang must be <= 65535 per call");
    if (!Y || !out) return fail(FCAT_E_INVALID_ARG, "Y and out must not be NULL");
    if ((s = check_pending())) return s;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PSF, static_cast<hipStream_t>(stream));
        e = launch_psf(Y, n_ang, n_groups, nv, nu, psf->kernels, psf->k, out, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return device_fail(e, "psf");
    return FCAT_OK;
}

fcat_status fcat_check_inputs(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                              const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                              const fcat_psf_t *psf, void *workspace, size_t workspace_bytes,
                              void *stream_)
{
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_phantom(phantom)) || (s = check_spectral(spectral, true, t)) || (s = check_psf(psf)))
        return s;
    if (scatter && (!geometry || check_geometry(geometry)))
        return fail(FCAT_E_INVALID_ARG, "a valid geometry is needed to check scatter maps");
    if ((s = check_workspace(workspace, workspace_bytes, 256))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    int *flags = static_cast<int *>(workspace);
    hipError_t e = launch_zero_ints(flags, 2, stream);
    const int64_t nvox = (int64_t)phantom->nx * phantom->ny * phantom->nz;
    if (e == hipSuccess) e = launch_check_labels(phantom->labels, nvox, t.M, flags, stream);
    const int E = t.E;
    if (e == hipSuccess) e = launch_check_finite(spectral->mu, (int64_t)t.M * E, flags + 1, stream);
    if (e == hipSuccess) e = launch_check_finite(spectral->phi, E, flags + 1, stream);
    if (e == hipSuccess) e = launch_check_finite(spectral->eta, E, flags + 1, stream);
    if (e == hipSuccess && spectral->flood && geometry && !check_geometry(geometry))
        e = launch_check_finite(spectral->flood, (int64_t)geometry->nu * geometry->nv, flags + 1, stream);
    if (e == hipSuccess && scatter) {
        if (scatter->maps)
            e = launch_check_finite(scatter->maps,
                                    (int64_t)geometry->n_angles * geometry->nu * geometry->nv, flags + 1,
                                    stream);
        if (e == hipSuccess && scatter->s_bin) e = launch_check_finite(scatter->s_bin, E, flags + 1, stream);
    }
    if (e == hipSuccess && psf)
        e = launch_check_finite(psf->kernels, (int64_t)t.G * psf->k * psf->k, flags + 1, stream);
    if (e != hipSuccess) return device_fail(e, "check kernels");
    int host[2] = {0, 0};
    e = hipMemcpyAsync(host, flags, sizeof host, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_fail(e, "check readback");
    if (host[0]) return fail(FCAT_E_LABEL_RANGE, "a phantom label is outside 0..%d", t.M - 1);
    if (host[1]) return fail(FCAT_E_NONFINITE, "a float table holds NaN or Inf");
    return FCAT_OK;
}

fcat_status fcat_timing_enable(int enable)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = enable != 0;
    return FCAT_OK;
}

fcat_status fcat_timing_read(double *ms, int64_t *launches, int32_t n_stages, int reset)
{
    g_last_error.clear();
    if (n_stages < 0) return fail(FCAT_E_INVALID_ARG, "n_stages must be >= 0");
    std::lock_guard<std::mutex> lk(g_tmu);
    for (int i = 0; i < n_stages; ++i) {
        if (ms) ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    for (const Timed &t : g_timed) {
        hipError_t e = hipEventSynchronize(t.b);
        float dt = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&dt, t.a, t.b);
        if (e != hipSuccess) return device_fail(e, "timing events");
        if (t.stage < n_stages) {
            if (ms) ms[t.stage] += dt;
            if (launches) launches[t.stage] += 1;
        }
    }
    if (reset) {
        for (const Timed &t : g_timed) {
            g_free_events.push_back(t.a);
            g_free_events.push_back(t.b);
        }
        g_timed.clear();
    }
    return FCAT_OK;
}

}  // extern "C"
