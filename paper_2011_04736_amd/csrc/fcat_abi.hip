// C ABI of libfcat.so: host-side argument validation, workspace layout,
// angle chunking and kernel launches.  See include/fcat.h for the contract.
#include "fcat_internal.h"
#include "fcat_recon.h"
#include "fcat_optics.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// Static scratch of fcat_spectral_static, for callers that cannot allocate
// device memory: its spectral tables live here instead of in a workspace.
// Each GPU holds its own copy of the array (at its own address) from the
// first call on it until the process ends.  In host code the array's name
// is not a device address; the address comes from hipGetSymbolAddress, once
// per device, and only that address is ever passed to a kernel.
static __device__ __align__(256) unsigned char scratch[2u << 20];

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
    auto bricks = [](int32_t n) { return ((int64_t)n + kBrickEdge - 1) / kBrickEdge; };   // 64-bit: n may be 2^31 - 1
    const int64_t bricked = bricks(p->nx) * bricks(p->ny) * bricks(p->nz) * kBrickVox;
    if (bricked + 2 * (int64_t)kLabelPad >= ((int64_t)1 << 31))
        return fail(FCAT_E_INVALID_ARG, "phantom rounded up to 16^3 bricks must hold fewer than 2^31 voxels");
    if (!finite_pos(p->dx_mm) || !finite_pos(p->dy_mm) || !finite_pos(p->dz_mm))
        return fail(FCAT_E_INVALID_ARG, "voxel sizes must be finite and > 0");
    if (!std::isfinite(p->cx_mm) || !std::isfinite(p->cy_mm) || !std::isfinite(p->cz_mm))
        return fail(FCAT_E_INVALID_ARG, "grid centre must be finite");
    return FCAT_OK;
}

// Material slots the kernels are compiled for: each spectral bin costs one
// FMA per slot, so the common counts get a close fit (10: the head phantom).
int padded_materials(int m) { return m <= 8 ? 8 : (m <= 10 ? 10 : (m <= 12 ? 12 : (m <= 16 ? 16 : 32))); }

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

// brick map + brick-major label copy with its padding
// The brick region of a workspace: brick map, background box (int[8]), padding,
// brick-major labels, padding.
constexpr size_t kClipBytes = 256;
size_t brick_bytes(const fcat_phantom_t *p)
{
    return align_up(brick_count(p)) + kClipBytes + brick_count(p) * kBrickVox + 2 * (size_t)kLabelPad;
}
// the background box, in a workspace whose brick map starts at `bricks`
int *clip_at(int8_t *bricks, const fcat_phantom_t *p) { return reinterpret_cast<int *>(bricks + align_up(brick_count(p))); }
// brick 0 of the brick-major labels
int8_t *labels_bm_at(int8_t *bricks, const fcat_phantom_t *p)
{
    return bricks + align_up(brick_count(p)) + kClipBytes + kLabelPad;
}

}  // namespace

int tile_log2u_for(const TraceGeom &G)
{
    // detector rows covered by the grid's z extent at the largest magnification
    // (grid corner nearest the source)
    const double rx = 0.5 * G.n[0] * G.h[0] + fabs(G.lo[0] + 0.5 * G.n[0] * G.h[0]);
    const double ry = 0.5 * G.n[1] * G.h[1] + fabs(G.lo[1] + 0.5 * G.n[1] * G.h[1]);
    const double near = G.sid - sqrt(rx * rx + ry * ry);
    const double mag = near > 0.0 ? (G.sid + G.back) / near : 1e9;
    const double rows = G.n[2] * G.h[2] * mag / G.dv;
    return rows < 24.0 ? 4 : 3;
}

namespace {

TraceGeom make_geom_box(const fcat_geometry_t *g, const int (&n)[3], const double (&h)[3], const double (&c)[3])
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
    G.trig = nullptr;
    for (int ax = 0; ax < 3; ++ax) G.nb[ax] = (n[ax] + kBrickEdge - 1) / kBrickEdge;
    G.bricks = nullptr;
    G.labels_bm = nullptr;
    G.clip = nullptr;
    G.tile_log2u = tile_log2u_for(G);
    return G;
}

TraceGeom make_geom(const fcat_geometry_t *g, const fcat_phantom_t *p)
{
    const int n[3] = {p->nx, p->ny, p->nz};
    const double h[3] = {p->dx_mm, p->dy_mm, p->dz_mm};
    const double c[3] = {p->cx_mm, p->cy_mm, p->cz_mm};
    return make_geom_box(g, n, h, c);
}

struct Layout {
    size_t flags, muT, w, Wg, Wsg, afrag, wtile, pfrag, frag, mbar, cslots, bricks, trig, Y, fixed;
    size_t scale, unitk, flood, yflood;   // projection stage: c_g, unit kernels, flood, its group signals
    size_t per_angle;    // bytes of per-angle chunk buffers (group signals)
    size_t y_per_angle;  // bytes of group signal per angle (0 without psf)
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
              const SplitTables *sp = nullptr, bool surrogate = false, int psf_split_k = 0, bool proj = false)
{
    Layout L{};
    size_t o = 0;
    L.flags = o;
    o += align_up(64 * sizeof(int));
    L.muT = o;
    o += align_up(2 * (size_t)t.E * t.mp * sizeof(float));   // mu, then mu log2(e)
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
    L.pfrag = o;
    if (psf_split_k > 0) o += align_up(psf_split_frag_count(t.G, psf_split_k) * 16);
    L.frag = o;
    if (surrogate) o += align_up((size_t)kMlpFrags * kWave * 16);
    L.mbar = o;
    if (surrogate) o += align_up((size_t)FCAT_MLP_MAX_IO * sizeof(float));
    L.cslots = o;   // ray counts of the surrogate projector, spread over slots
    if (surrogate) o += align_up((size_t)kCountSlots * kCountSlotInts * sizeof(int));
    L.bricks = o;
    o += align_up(nbricks);
    L.trig = o;   // cosine and sine of every angle
    if (g) o += align_up((size_t)g->n_angles * 2 * sizeof(double));
    const size_t plane = g ? (size_t)g->nu * g->nv : 0;
    L.scale = o;
    if (proj) o += align_up((size_t)t.G * sizeof(float));
    L.unitk = o;
    if (proj) o += align_up((size_t)t.G * sizeof(float));
    L.flood = o;
    if (proj) o += align_up(plane * sizeof(float));
    L.yflood = o;
    if (proj) o += align_up((size_t)t.G * plane * sizeof(float));
    L.fixed = o;
    L.y_per_angle = (with_psf && g) ? align_up((size_t)t.G * g->nu * g->nv * sizeof(float)) : 0;
    L.per_angle = L.y_per_angle;
    L.Y = o;       // the chunk buffer follows the fixed part: Y [chunk][G][plane]
    return L;
}

constexpr size_t kDefaultChunkBytes = (size_t)1 << 30;
// Projector chunks when the job does not fit in one: measured on the head
// workload (25 MB of group signals per angle), 16 angles per launch took
// 87.5 ms per step, 32 took 89.0, 40 (1 GiB) 92.0 and 8 88.3 (later, with a
// faster walk: 16 and 8 84.6 and 84.7, 24 86.0).  On the
// contrast workload (2 MiB per angle) one launch for all 360 angles is best
// (2.10 ms; 2.29 ms in chunks of 90).
constexpr size_t kProjectChunkBytes = (size_t)384 << 20;

// Angles per chunk when the caller leaves the choice to the library: all of
// them in one launch if their chunk buffers fit in kDefaultChunkBytes, else
// as many as fit in kProjectChunkBytes.
int default_chunk(const Layout &L, int n_angles)
{
    if (L.per_angle == 0) return n_angles;
    if ((size_t)n_angles * L.per_angle <= kDefaultChunkBytes) return n_angles;
    size_t c = kProjectChunkBytes / L.per_angle;
    // a multiple of the XCD count when there is room: on the head workload
    // 8 and 16 angles per launch took 84.7 and 84.6 ms per step, 10, 12 and
    // 20 took 96.5, 88.3 and 87.0
    if (c >= (size_t)kXcds) c -= c % kXcds;
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

// ------------------------------------------------------------ static scratch

constexpr size_t kStaticScratchBytes = sizeof(scratch);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_at[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
fcat_status static_scratch(void **addr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FCAT_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (uintptr_t)p % kAlign) return fail(FCAT_E_DEVICE, "static scratch at an unusable address");
        g_scratch_at[dev] = p;
    }
    *addr = g_scratch_at[dev];
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
                        void *ws, hipStream_t stream, const InputCheck &chk = InputCheck())
{
    float *muT = at<float>(ws, L.muT), *w = at<float>(ws, L.w);
    float *Wg = at<float>(ws, L.Wg), *Wsg = at<float>(ws, L.Wsg);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        e = launch_prep_tables(s->mu, s->phi, s->eta, s_bin, t, muT, w, Wg, Wsg, stream, chk);
    }
    if (e != hipSuccess) return device_fail(e, "prep_tables");
    t.muT = muT;
    t.mu2T = muT + (size_t)t.E * t.mp;
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

fcat_status check_surrogate(const fcat_surrogate_t *u, const SpecTables &t, bool need_cells)
{
    if (!u) return fail(FCAT_E_INVALID_ARG, "surrogate is NULL");
    if (u->n_in != t.M || u->n_out != t.G)
        return fail(FCAT_E_INVALID_ARG, "surrogate n_in/n_out must equal n_mat/n_groups");
    if (u->n_in < 1 || u->n_in > FCAT_MLP_MAX_IO || u->n_out < 1 || u->n_out > FCAT_MLP_MAX_IO)
        return fail(FCAT_E_INVALID_ARG, "surrogate n_in and n_out must be in 1..%d", FCAT_MLP_MAX_IO);
    if (!u->params || !u->in_scale || !u->out_scale || !u->lin)
        return fail(FCAT_E_INVALID_ARG, "surrogate params, in_scale, out_scale and lin must not be NULL");
    if (need_cells) {
        if (!u->cell_ok) return fail(FCAT_E_INVALID_ARG, "surrogate cell_ok is NULL");
        if (!std::isfinite(u->cell_lo) || !std::isfinite(u->cell_hi) || !(u->cell_lo < u->cell_hi))
            return fail(FCAT_E_INVALID_ARG, "surrogate cell range must be finite with cell_lo < cell_hi");
    }
    return FCAT_OK;
}

fcat_status prep_mlp(const fcat_surrogate_t *u, const float *params, const SpecTables &t, const Layout &L, void *ws,
                     hipStream_t stream, MlpTables &mt)
{
    uint4 *frag = at<uint4>(ws, L.frag);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        e = launch_mlp_prep(params, t.M, t.G, frag, stream);
    }
    float *mbar = at<float>(ws, L.mbar);
    if (e == hipSuccess) e = launch_mlp_mbar(t, u->lin, mbar, stream);
    if (e != hipSuccess) return device_fail(e, "mlp_prep");
    mt.frag = frag;
    mt.mbar = mbar;
    mt.params = params;
    mt.in_scale = u->in_scale;
    mt.out_scale = u->out_scale;
    mt.lin = u->lin;
    mt.cell_ok = u->cell_ok;
    mt.cell_lo = u->cell_lo;
    mt.cell_hi = u->cell_hi;
    mt.n_in = t.M;
    mt.n_out = t.G;
    return FCAT_OK;
}

// Workspace of the fcat_mlp_* calls: spectral tables, fragments, per-wave
// gradient partials and loss sums, and the validation cells.
struct MlpLayout {
    Layout base;
    size_t partial, loss_partial, cells, stats, fcnt, finv, total;
    int nparts, P;
};

MlpLayout mlp_layout(const SpecTables &t, int64_t batch)
{
    MlpLayout m{};
    m.base = layout(t, nullptr, false, 0, nullptr, true);
    m.P = mlp_param_count(t.M, t.G);
    m.nparts = (int)((std::max<int64_t>(batch, 1) + kWave - 1) / kWave);
    size_t o = m.base.fixed;
    m.partial = o;
    o += align_up((size_t)m.nparts * m.P * sizeof(float));
    m.loss_partial = o;
    o += align_up((size_t)m.nparts * sizeof(float));
    m.cells = o;
    o += align_up((size_t)2 * FCAT_MLP_MAX_IO * FCAT_MLP_CELLS * sizeof(int));
    m.stats = o;
    o += align_up((size_t)kStatBlocks * kStatStride * sizeof(float));
    m.fcnt = o;   // fragment elements per parameter (training)
    o += align_up((size_t)m.P * sizeof(int));
    m.finv = o;
    o += align_up((size_t)m.P * kMlpViews * sizeof(uint32_t));
    m.total = o;
    return m;
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

// k of the matrix-core optical spread in the split form, or 0 where the FP32 one runs.
static int psf_split_k(const fcat_psf_t *psf, fcat_mode mode)
{
    return (psf && mode == FCAT_MODE_SPLIT_BF16 && psf->k <= kPsfSplitMaxK) ? psf->k : 0;
}

// Workspace of the projector; proj adds the projection stage, noisy the
// group signals it needs even without the optical spread.
static size_t project_ws_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                               const fcat_spectral_t *spectral, const fcat_psf_t *psf, fcat_mode mode,
                               int32_t angles_per_chunk, bool proj, bool noisy)
{
    SpecTables t{};
    if (check_geometry(geometry) || check_phantom(phantom) || check_spectral(spectral, false, t) ||
        check_psf(psf))
        return 0;
    SplitTables sp{};
    split_host(t, sp);
    Layout L = layout(t, geometry, psf != nullptr || noisy, brick_bytes(phantom),
                      mode == FCAT_MODE_SPLIT_BF16 ? &sp : nullptr, mode == FCAT_MODE_SURROGATE,
                      psf_split_k(psf, mode), proj);
    int chunk = angles_per_chunk > 0 ? angles_per_chunk : default_chunk(L, geometry->n_angles);
    if (chunk > geometry->n_angles) chunk = geometry->n_angles;
    return L.fixed + (size_t)chunk * L.per_angle;
}

size_t fcat_project_workspace_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                    const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                                    const fcat_psf_t *psf, fcat_mode mode, int32_t angles_per_chunk)
{
    (void)scatter;
    return project_ws_bytes(geometry, phantom, spectral, psf, mode, angles_per_chunk, false, false);
}

size_t fcat_projections_workspace_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                        const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                                        const fcat_psf_t *psf, fcat_mode mode, int32_t angles_per_chunk)
{
    (void)scatter;
    // sized for the noisy case, which needs the most
    return project_ws_bytes(geometry, phantom, spectral, psf, mode, angles_per_chunk, true, true);
}

static fcat_status check_noise(const fcat_noise_t *n)
{
    if (!n) return FCAT_OK;
    if (!(n->counts_per_pixel > 0.0) || !std::isfinite(n->counts_per_pixel))
        return fail(FCAT_E_INVALID_ARG, "counts_per_pixel must be finite and > 0");
    if (!(n->floor >= 0.0f) || !std::isfinite(n->floor)) return fail(FCAT_E_INVALID_ARG, "floor must be finite and >= 0");
    return FCAT_OK;
}

// The projector (fcat_project) and, with proj, the noise and projection
// stage after it (fcat_projections): out then receives projections.
static fcat_status project_impl(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                                const fcat_psf_t *psf, fcat_mode mode, const fcat_surrogate_t *surrogate,
                                bool proj, const fcat_noise_t *noise, float *out, void *workspace,
                                size_t workspace_bytes, void *stream_)
{
    SpecTables t{};
    fcat_status s;
    if ((s = check_geometry(geometry)) || (s = check_phantom(phantom)) ||
        (s = check_spectral(spectral, true, t)) || (s = check_psf(psf)) || (s = check_noise(noise)))
        return s;
    if (!out) return fail(FCAT_E_INVALID_ARG, "output is NULL");
    if (scatter && !scatter->maps) return fail(FCAT_E_INVALID_ARG, "scatter maps is NULL");
    if (mode != FCAT_MODE_PLAIN && mode != FCAT_MODE_SPLIT_BF16 && mode != FCAT_MODE_SURROGATE)
        return fail(FCAT_E_INVALID_ARG, "unknown mode %d", (int)mode);
    const bool split = mode == FCAT_MODE_SPLIT_BF16;
    const bool sur = mode == FCAT_MODE_SURROGATE;
    const bool noisy = proj && noise != nullptr;
    const bool grouped = psf != nullptr || noisy;   // group signals pass through the workspace
    if (sur && (s = check_surrogate(surrogate, t, true))) return s;
    const int64_t plane = (int64_t)geometry->nu * geometry->nv;
    if (proj && plane >= ((int64_t)1 << 31)) return fail(FCAT_E_INVALID_ARG, "nu * nv must be < 2^31");
    SplitTables sp{};
    split_host(t, sp);
    const int pk = psf_split_k(psf, mode);
    Layout L = layout(t, geometry, grouped, brick_bytes(phantom), split ? &sp : nullptr, sur, pk, proj);
    const size_t need = L.fixed + L.per_angle;  // at least one angle per chunk
    if ((s = check_workspace(workspace, workspace_bytes, need))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);

    // input problems found on the way (see fcat_project_status): cleared here,
    // set by the kernels that read each input anyway
    int *bad = at<int>(workspace, L.flags);
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        hipError_t e0 = launch_zero_ints(bad, kInputFlags, stream);
        if (e0 != hipSuccess) return device_fail(e0, "clear input flags");
    }
    InputCheck chk;
    chk.bad = bad;
    chk.psf = psf ? psf->kernels : nullptr;
    chk.n_psf = psf ? t.G * psf->k * psf->k : 0;
    if ((s = prep_tables(spectral, scatter ? scatter->s_bin : nullptr, t, L, workspace, stream, chk))) return s;
    if (split && (s = prep_split(spectral, t, sp, L, workspace, stream))) return s;
    uint4 *pfrag = at<uint4>(workspace, L.pfrag);
    if (pk) {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        hipError_t e0 = launch_prep_psf_split(psf->kernels, t.G, pk, pfrag, stream);
        if (e0 != hipSuccess) return device_fail(e0, "prep_psf_split");
    }
    MlpTables mt{};
    if (sur && (s = prep_mlp(surrogate, surrogate->params, t, L, workspace, stream, mt))) return s;
    TraceGeom G = make_geom(geometry, phantom);
    G.bricks = at<int8_t>(workspace, L.bricks);
    G.labels_bm = labels_bm_at(const_cast<int8_t *>(G.bricks), phantom);
    G.bad = bad;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        int *clip = clip_at(const_cast<int8_t *>(G.bricks), phantom);
        hipError_t e0 = launch_build_bricks(phantom->labels, phantom->nx, phantom->ny, phantom->nz,
                                            const_cast<int8_t *>(G.bricks), const_cast<int8_t *>(G.labels_bm), clip,
                                            stream, t.M, bad);
        G.clip = clip;
        if (e0 != hipSuccess) return device_fail(e0, "build_bricks");
        e0 = launch_trig_table(G, at<double>(workspace, L.trig), stream);
        if (e0 != hipSuccess) return device_fail(e0, "trig_table");
        G.trig = at<double>(workspace, L.trig);
    }
    const float *S = scatter ? scatter->maps : nullptr;
    const int A = geometry->n_angles;
    hipError_t e;
    int *cslots = (sur && surrogate->counts) ? at<int>(workspace, L.cslots) : nullptr;
    if (cslots) {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        e = launch_zero_ints(cslots, kCountSlots * kCountSlotInts, stream);
        if (e != hipSuccess) return device_fail(e, "clear count slots");
    }
    // the slots' totals into the caller's counters, after the last walk (timed
    // with the set-up, so that the walk's stage holds one launch per chunk)
    auto add_counts = [&]() -> hipError_t {
        if (!cslots) return hipSuccess;
        StageTimer tm(FCAT_STAGE_PREP, stream);
        return launch_count_slots_sum(cslots, surrogate->counts, stream);
    };
    float *unitk = at<float>(workspace, L.unitk);
    // optical spread and group sum of n angles of group signals (unit kernels without psf)
    auto spread = [&](const float *Yc, int n, float *dst) {
        StageTimer tm(FCAT_STAGE_PSF, stream);
        if (pk) return launch_psf_split(Yc, n, t.G, geometry->nv, geometry->nu, pk, pfrag, dst, stream);
        return launch_psf(Yc, n, t.G, geometry->nv, geometry->nu, psf ? psf->kernels : unitk, psf ? psf->k : 1, dst,
                          stream);
    };
    float *scale = at<float>(workspace, L.scale);
    float *flood = at<float>(workspace, L.flood);
    const float floor_ = noise ? noise->floor : 0.0f;
    if (proj) {
        {
            StageTimer tm(FCAT_STAGE_PROJ, stream);
            e = noisy ? launch_count_scale(spectral->phi, spectral->eta, t.gstart, t.E, t.G, noise->counts_per_pixel,
                                           scale, stream)
                      : hipSuccess;
            if (e == hipSuccess && !psf) e = launch_fill(unitk, t.G, 1.0f, stream);
            if (e == hipSuccess)
                e = launch_flood_groups(t.Wg, spectral->flood, plane, t.G, at<float>(workspace, L.yflood), stream);
        }
        if (e == hipSuccess) e = spread(at<float>(workspace, L.yflood), 1, flood);
        if (e != hipSuccess) return device_fail(e, "flood profile");
    }
    auto to_projections = [&](float *o, int n) {
        StageTimer tm(FCAT_STAGE_PROJ, stream);
        return launch_log_projection(o, flood, n, plane, floor_, o, stream);
    };
    auto rows = [&](int a0, int n, float *Yc, float *outc) {
        if (sur)
            return launch_project_rows_mlp(G, t, mt, spectral->flood, S, a0, n, Yc, outc, cslots, stream);
        return split ? launch_project_rows_split(G, phantom->labels, t, sp, spectral->flood, S, a0, n, Yc, outc, stream)
                     : launch_project_rows(G, phantom->labels, t, spectral->flood, S, a0, n, Yc, outc, stream);
    };
    if (L.per_angle == 0) {
        {
            StageTimer tm(FCAT_STAGE_TRACE, stream);
            e = rows(0, A, nullptr, out);
        }
        if (e != hipSuccess) return device_fail(e, "project_rows");
        if ((e = add_counts()) != hipSuccess) return device_fail(e, "count_slots_sum");
        if (proj && (e = to_projections(out, A)) != hipSuccess) return device_fail(e, "log_projection");
        return FCAT_OK;
    }
    const int chunk = (int)std::min<size_t>((size_t)A, (workspace_bytes - L.fixed) / L.per_angle);
    float *Y = grouped ? at<float>(workspace, L.Y) : nullptr;
    for (int a0 = 0; a0 < A; a0 += chunk) {
        const int n = std::min(chunk, A - a0);
        float *outc = out + a0 * plane;
        {
            StageTimer tm(FCAT_STAGE_TRACE, stream);
            e = rows(a0, n, Y, grouped ? nullptr : outc);
            if (e != hipSuccess) return device_fail(e, "project_rows");
        }
        if (noisy) {
            StageTimer tm(FCAT_STAGE_NOISE, stream);
            e = launch_poisson(Y, n, t.G, plane, scale, noise->seed, a0, stream);
            if (e != hipSuccess) return device_fail(e, "poisson");
        }
        if (grouped && (e = spread(Y, n, outc)) != hipSuccess) return device_fail(e, "psf");
        if (proj && (e = to_projections(outc, n)) != hipSuccess) return device_fail(e, "log_projection");
    }
    if ((e = add_counts()) != hipSuccess) return device_fail(e, "count_slots_sum");
    return FCAT_OK;
}

fcat_status fcat_project(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                         const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                         const fcat_psf_t *psf, fcat_mode mode, const fcat_surrogate_t *surrogate,
                         float *out, void *workspace, size_t workspace_bytes, void *stream)
{
    g_last_error.clear();
    return project_impl(geometry, phantom, spectral, scatter, psf, mode, surrogate, false, nullptr, out, workspace,
                        workspace_bytes, stream);
}

fcat_status fcat_project_status(const void *workspace, size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    fcat_status s;
    if ((s = check_workspace(const_cast<void *>(workspace), workspace_bytes, kAlign))) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    int host[kInputFlags] = {0, 0};
    hipError_t e = hipMemcpyAsync(host, workspace, sizeof host, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_fail(e, "input flags readback");
    if (host[0]) return fail(FCAT_E_LABEL_RANGE, "a phantom label is outside 0..n_mat-1 (those voxels added no path length)");
    if (host[1]) return fail(FCAT_E_NONFINITE, "mu, phi, eta, s_bin, flood, scatter or a spread kernel holds NaN or Inf");
    return FCAT_OK;
}

fcat_status fcat_projections(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                             const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                             const fcat_psf_t *psf, fcat_mode mode, const fcat_surrogate_t *surrogate,
                             const fcat_noise_t *noise, float *proj, void *workspace, size_t workspace_bytes,
                             void *stream)
{
    g_last_error.clear();
    return project_impl(geometry, phantom, spectral, scatter, psf, mode, surrogate, true, noise, proj, workspace,
                        workspace_bytes, stream);
}

// Workspace of fcat_dose: tables and bricks, then S [E], the workgroup
// partials, and the path lengths of a chunk of angles.
struct DoseLayout {
    Layout base;
    size_t S, partial, L, fixed, per_angle;
};

static DoseLayout dose_layout(const SpecTables &t, const fcat_geometry_t *g, const fcat_phantom_t *p)
{
    DoseLayout d{};
    d.base = layout(t, nullptr, false, brick_bytes(p));
    size_t o = d.base.fixed;
    d.S = o;
    o += align_up((size_t)t.E * sizeof(double));
    d.partial = o;
    o += align_up((size_t)kDoseBlocks * t.E * sizeof(double));
    d.L = o;
    d.fixed = o;
    d.per_angle = (size_t)g->nu * g->nv * t.M * sizeof(float);
    return d;
}

size_t fcat_dose_workspace_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                 const fcat_spectral_t *spectral, int32_t angles_per_chunk)
{
    SpecTables t{};
    if (check_geometry(geometry) || check_phantom(phantom) || check_spectral(spectral, false, t)) return 0;
    const DoseLayout d = dose_layout(t, geometry, phantom);
    size_t chunk = angles_per_chunk > 0 ? (size_t)angles_per_chunk : kDefaultChunkBytes / d.per_angle;
    chunk = std::max<size_t>(1, std::min<size_t>(chunk, (size_t)geometry->n_angles));
    return d.fixed + align_up(chunk * d.per_angle);
}

fcat_status fcat_dose(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                      const fcat_spectral_t *spectral, const float *energy, const float *mu_en_over_mu,
                      double mass, int32_t a_begin, int32_t a_end, double *D0, double *Dp, void *workspace,
                      size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_geometry(geometry)) || (s = check_phantom(phantom)) || (s = check_spectral(spectral, true, t)))
        return s;
    if (!energy || !mu_en_over_mu || !D0) return fail(FCAT_E_INVALID_ARG, "energy, mu_en_over_mu and D0 must not be NULL");
    if (!(mass > 0.0) || !std::isfinite(mass)) return fail(FCAT_E_INVALID_ARG, "mass must be finite and > 0");
    if (a_begin < 0 || a_end > geometry->n_angles || a_begin >= a_end)
        return fail(FCAT_E_INVALID_ARG, "need 0 <= a_begin < a_end <= n_angles");
    const DoseLayout d = dose_layout(t, geometry, phantom);
    if ((s = check_workspace(workspace, workspace_bytes, d.fixed + align_up(d.per_angle)))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((s = prep_tables(spectral, nullptr, t, d.base, workspace, stream))) return s;
    TraceGeom G = make_geom(geometry, phantom);
    G.bricks = at<int8_t>(workspace, d.base.bricks);
    G.labels_bm = labels_bm_at(const_cast<int8_t *>(G.bricks), phantom);
    double *S = at<double>(workspace, d.S);
    double *partial = at<double>(workspace, d.partial);
    float *L = at<float>(workspace, d.L);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        G.clip = clip_at(const_cast<int8_t *>(G.bricks), phantom);
        e = launch_build_bricks(phantom->labels, phantom->nx, phantom->ny, phantom->nz,
                                const_cast<int8_t *>(G.bricks), const_cast<int8_t *>(G.labels_bm),
                                const_cast<int *>(G.clip), stream);
        if (e == hipSuccess) e = launch_zero_doubles(S, t.E, stream);
    }
    if (e != hipSuccess) return device_fail(e, "dose set-up");
    const int64_t plane = (int64_t)geometry->nu * geometry->nv;
    const int chunk = (int)std::min<size_t>((size_t)(a_end - a_begin), (workspace_bytes - d.fixed) / d.per_angle);
    for (int a0 = a_begin; a0 < a_end; a0 += chunk) {
        const int n = std::min(chunk, a_end - a0);
        {
            StageTimer tm(FCAT_STAGE_TRACE, stream);
            e = launch_pathlengths(G, phantom->labels, t.M, a0, n, L, stream);
        }
        if (e != hipSuccess) return device_fail(e, "pathlengths");
        const int64_t rays = (int64_t)n * plane;
        {
            StageTimer tm(FCAT_STAGE_DOSE, stream);
            e = launch_dose_rays(L, rays, t.M, t, partial, stream);
            if (e == hipSuccess) e = launch_dose_sum(partial, dose_blocks(rays), t.E, S, stream);
        }
        if (e != hipSuccess) return device_fail(e, "dose sums");
    }
    const double n_rays = (double)(a_end - a_begin) * (double)plane;
    {
        StageTimer tm(FCAT_STAGE_DOSE, stream);
        e = launch_dose_final(S, energy, mu_en_over_mu, spectral->phi, t.E, 1.0 / (n_rays * mass), D0, Dp, stream);
    }
    if (e != hipSuccess) return device_fail(e, "dose");
    return FCAT_OK;
}

// ------------------------------------------------------------------ FDK

static FdkGeom fdk_geom(const fcat_geometry_t *g)
{
    FdkGeom f{};
    f.D = (float)g->sid_mm;
    f.scale = (float)(g->sdd_mm / g->sid_mm);
    f.du = (float)g->du_mm;
    f.dv = (float)g->dv_mm;
    f.off_u = (float)g->off_u_mm;
    f.off_v = (float)g->off_v_mm;
    f.cu = 0.5f * (float)(g->nu - 1);
    f.cv = 0.5f * (float)(g->nv - 1);
    f.tau = (float)(g->du_mm * g->sid_mm / g->sdd_mm);
    f.inv_du = (float)(1.0 / g->du_mm);
    f.inv_dv = (float)(1.0 / g->dv_mm);
    f.nu = g->nu;
    f.nv = g->nv;
    return f;
}

static fcat_status check_grid(const fcat_grid_t *v, FdkGrid &out)
{
    if (!v) return fail(FCAT_E_INVALID_ARG, "grid is NULL");
    if (v->nx < 1 || v->ny < 1 || v->nz < 1) return fail(FCAT_E_INVALID_ARG, "grid nx, ny, nz must be >= 1");
    if ((int64_t)v->nx * v->ny * v->nz >= ((int64_t)1 << 31))
        return fail(FCAT_E_INVALID_ARG, "grid larger than 2^31 - 1 voxels");
    if (!finite_pos(v->dx_mm) || !finite_pos(v->dy_mm) || !finite_pos(v->dz_mm))
        return fail(FCAT_E_INVALID_ARG, "grid voxel sizes must be finite and > 0");
    if (!std::isfinite(v->cx_mm) || !std::isfinite(v->cy_mm) || !std::isfinite(v->cz_mm))
        return fail(FCAT_E_INVALID_ARG, "grid centre must be finite");
    out.x0 = (float)(v->cx_mm - 0.5 * v->nx * v->dx_mm + 0.5 * v->dx_mm);
    out.y0 = (float)(v->cy_mm - 0.5 * v->ny * v->dy_mm + 0.5 * v->dy_mm);
    out.z0 = (float)(v->cz_mm - 0.5 * v->nz * v->dz_mm + 0.5 * v->dz_mm);
    out.dx = (float)v->dx_mm;
    out.dy = (float)v->dy_mm;
    out.dz = (float)v->dz_mm;
    out.nx = v->nx;
    out.ny = v->ny;
    out.nz = v->nz;
    return FCAT_OK;
}

// Widest detector row the ramp filter's workgroup holds in LDS: 7704 columns.
static bool fdk_nu_supported(int nu) { return fdk_filter_lds_bytes(nu) <= kFdkFilterMaxLds; }

fcat_status fcat_fdk_filter(const fcat_geometry_t *geometry, const float *proj, int32_t n_ang, float *filtered,
                            void *stream)
{
    g_last_error.clear();
    fcat_status s;
    if ((s = check_geometry(geometry))) return s;
    if (!fdk_nu_supported(geometry->nu))
        return fail(FCAT_E_UNSUPPORTED, "the FDK filter takes nu <= 7704 (its rows are held in 64 KiB of LDS)");
    if (n_ang < 1) return fail(FCAT_E_INVALID_ARG, "n_ang must be >= 1");
    if (!proj || !filtered) return fail(FCAT_E_INVALID_ARG, "proj and filtered must not be NULL");
    const size_t bytes = (size_t)n_ang * geometry->nv * geometry->nu * sizeof(float);
    const char *p0 = reinterpret_cast<const char *>(proj), *f0 = reinterpret_cast<const char *>(filtered);
    if (p0 < f0 + bytes && f0 < p0 + bytes) return fail(FCAT_E_INVALID_ARG, "proj and filtered overlap");
    if ((s = check_pending())) return s;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_FILTER, static_cast<hipStream_t>(stream));
        e = launch_fdk_filter(fdk_geom(geometry), proj, n_ang, false, filtered, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return device_fail(e, "fdk_filter");
    return FCAT_OK;
}

size_t fcat_fdk_backproject_workspace_bytes(int32_t n_ang)
{
    return n_ang < 1 ? 0 : align_up((size_t)n_ang * sizeof(float2));
}

static fcat_status fdk_backproject(const fcat_geometry_t *geometry, const float *filtered, const float4 *quads,
                                   int a_begin, int a_end, const FdkGrid &v, float *volume, int accumulate,
                                   float2 *cs, hipStream_t stream)
{
    const int n = a_end - a_begin;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_BACKPROJECT, stream);
        e = launch_fdk_angles(geometry->angles_rad, geometry->n_angles, a_begin, n, cs, stream);
        if (e == hipSuccess)
            e = launch_fdk_backproject(fdk_geom(geometry), v, filtered, quads, cs, n,
                                       (float)(3.141592653589793 / geometry->n_angles), accumulate, volume, stream);
    }
    if (e != hipSuccess) return device_fail(e, "fdk_backproject");
    return FCAT_OK;
}

fcat_status fcat_fdk_backproject(const fcat_geometry_t *geometry, const float *filtered, int32_t a_begin,
                                 int32_t a_end, const fcat_grid_t *grid, float *volume, int32_t accumulate,
                                 void *workspace, size_t workspace_bytes, void *stream)
{
    g_last_error.clear();
    fcat_status s;
    FdkGrid v{};
    if ((s = check_geometry(geometry)) || (s = check_grid(grid, v))) return s;
    if (a_begin < 0 || a_end > geometry->n_angles || a_begin >= a_end)
        return fail(FCAT_E_INVALID_ARG, "need 0 <= a_begin < a_end <= n_angles");
    if (!filtered || !volume) return fail(FCAT_E_INVALID_ARG, "filtered and volume must not be NULL");
    if ((s = check_workspace(workspace, workspace_bytes, fcat_fdk_backproject_workspace_bytes(a_end - a_begin))))
        return s;
    if ((s = check_pending())) return s;
    return fdk_backproject(geometry, filtered, nullptr, a_begin, a_end, v, volume, accumulate ? 1 : 0,
                           static_cast<float2 *>(workspace), static_cast<hipStream_t>(stream));
}

// bytes of one angle's filtered rows in fcat_fdk: the padded plane and its quads
static size_t fdk_padded_bytes(const fcat_geometry_t *g)
{
    return (size_t)fdk_padded_plane(g->nu, g->nv) * sizeof(float);
}
static size_t fdk_quad_bytes(const fcat_geometry_t *g)
{
    return (size_t)fdk_quad_plane(g->nu, g->nv) * sizeof(float4);
}
static size_t fdk_chunk_bytes(const fcat_geometry_t *g, size_t c)
{
    return align_up(c * fdk_padded_bytes(g)) + align_up(c * fdk_quad_bytes(g));
}

static size_t fdk_chunk(const fcat_geometry_t *g, int32_t angles_per_chunk)
{
    const size_t per = fdk_padded_bytes(g) + fdk_quad_bytes(g);
    size_t c = angles_per_chunk > 0 ? (size_t)angles_per_chunk : kDefaultChunkBytes / per;
    return std::max<size_t>(1, std::min<size_t>(c, (size_t)g->n_angles));
}

size_t fcat_fdk_workspace_bytes(const fcat_geometry_t *geometry, int32_t angles_per_chunk)
{
    if (check_geometry(geometry)) return 0;
    const size_t c = fdk_chunk(geometry, angles_per_chunk);
    return align_up((size_t)geometry->n_angles * sizeof(float2)) + fdk_chunk_bytes(geometry, c);
}

fcat_status fcat_fdk(const fcat_geometry_t *geometry, const float *proj, const fcat_grid_t *grid, float *volume,
                     void *workspace, size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    fcat_status s;
    FdkGrid v{};
    if ((s = check_geometry(geometry)) || (s = check_grid(grid, v))) return s;
    if (!fdk_nu_supported(geometry->nu))
        return fail(FCAT_E_UNSUPPORTED, "the FDK filter takes nu <= 7704 (its rows are held in 64 KiB of LDS)");
    if (!proj || !volume) return fail(FCAT_E_INVALID_ARG, "proj and volume must not be NULL");
    // the back-projection addresses an angle's quads with 32-bit offsets
    if (fdk_quad_bytes(geometry) >= ((size_t)1 << 32))
        return fail(FCAT_E_UNSUPPORTED, "FDK takes detectors with (nv + 2) (max(nu, 2) - 1) < 2^28");
    const size_t cs_bytes = align_up((size_t)geometry->n_angles * sizeof(float2));
    if ((s = check_workspace(workspace, workspace_bytes, cs_bytes + fdk_chunk_bytes(geometry, 1)))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    float2 *cs = static_cast<float2 *>(workspace);
    float *filt = at<float>(workspace, cs_bytes);
    const int A = geometry->n_angles;
    // the most angles whose padded planes and quads fit
    const size_t room = workspace_bytes - cs_bytes;
    size_t c = std::min<size_t>((size_t)A, room / (fdk_padded_bytes(geometry) + fdk_quad_bytes(geometry)));
    c = std::max<size_t>(c, 1);
    while (c > 1 && fdk_chunk_bytes(geometry, c) > room) --c;
    const int chunk = (int)c;
    float4 *quads = at<float4>(workspace, cs_bytes + align_up(c * fdk_padded_bytes(geometry)));
    const FdkGeom g = fdk_geom(geometry);
    // the filter writes only the rows of the detector: the zero pads of the
    // chunk buffer are written once and stay
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_LAYOUT, stream);
        e = launch_fdk_pad(g, chunk, filt, stream);
    }
    if (e != hipSuccess) return device_fail(e, "fdk_pad");
    for (int a0 = 0; a0 < A; a0 += chunk) {
        const int n = std::min(chunk, A - a0);
        {
            StageTimer tm(FCAT_STAGE_FILTER, stream);
            e = launch_fdk_filter(g, proj + (int64_t)a0 * geometry->nu * geometry->nv, n, true, filt, stream);
        }
        if (e != hipSuccess) return device_fail(e, "fdk_filter");
        {
            StageTimer tm(FCAT_STAGE_LAYOUT, stream);
            e = launch_fdk_quads(g, n, filt, quads, stream);
        }
        if (e != hipSuccess) return device_fail(e, "fdk_quads");
        if ((s = fdk_backproject(geometry, nullptr, quads, a0, a0 + n, v, volume, a0 > 0, cs, stream))) return s;
    }
    return FCAT_OK;
}

// ------------------------------------------------- image projector pair

static fcat_status image_args(const fcat_geometry_t *geometry, const fcat_grid_t *grid, int32_t a_begin,
                              int32_t a_end, const void *in, const void *out, TraceGeom &G)
{
    fcat_status s;
    FdkGrid fg;
    if ((s = check_geometry(geometry)) || (s = check_grid(grid, fg))) return s;
    if (a_begin < 0 || a_end > geometry->n_angles || a_begin >= a_end)
        return fail(FCAT_E_INVALID_ARG, "need 0 <= a_begin < a_end <= n_angles");
    if (!in || !out) return fail(FCAT_E_INVALID_ARG, "input and output must not be NULL");
    const int n[3] = {grid->nx, grid->ny, grid->nz};
    const double h[3] = {grid->dx_mm, grid->dy_mm, grid->dz_mm};
    const double c[3] = {grid->cx_mm, grid->cy_mm, grid->cz_mm};
    G = make_geom_box(geometry, n, h, c);
    return check_pending();
}

fcat_status fcat_image_project(const fcat_geometry_t *geometry, const fcat_grid_t *grid, const float *image,
                               int32_t a_begin, int32_t a_end, float *proj, void *stream_)
{
    g_last_error.clear();
    TraceGeom G;
    fcat_status s;
    if ((s = image_args(geometry, grid, a_begin, a_end, image, proj, G))) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_TRACE, stream);
        e = launch_image_project(G, image, a_begin, a_end - a_begin, proj, stream);
    }
    if (e != hipSuccess) return device_fail(e, "image_project");
    return FCAT_OK;
}

fcat_status fcat_image_backproject(const fcat_geometry_t *geometry, const fcat_grid_t *grid, const float *proj,
                                   int32_t a_begin, int32_t a_end, float *image, int32_t accumulate, void *stream_)
{
    g_last_error.clear();
    TraceGeom G;
    fcat_status s;
    if ((s = image_args(geometry, grid, a_begin, a_end, proj, image, G))) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipError_t e = hipSuccess;
    {
        StageTimer tm(FCAT_STAGE_BACKPROJECT, stream);
        if (!accumulate) e = launch_fill(image, grid->nx * grid->ny * grid->nz, 0.0f, stream);
        if (e == hipSuccess) e = launch_image_backproject(G, proj, a_begin, a_end - a_begin, image, stream);
    }
    if (e != hipSuccess) return device_fail(e, "image_backproject");
    return FCAT_OK;
}

// ------------------------------------------------------------ optics

fcat_status fcat_effective_psf(const fcat_spectral_t *spectral, const fcat_psf_t *psf, float *kernel, void *stream)
{
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_spectral(spectral, false, t))) return s;
    if (!psf) return fail(FCAT_E_INVALID_ARG, "psf is NULL");
    if ((s = check_psf(psf))) return s;
    if (!spectral->phi || !spectral->eta || !kernel) return fail(FCAT_E_INVALID_ARG, "phi, eta and kernel must not be NULL");
    if ((s = check_pending())) return s;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_OPTICS, static_cast<hipStream_t>(stream));
        e = launch_effective_psf(spectral->phi, spectral->eta, t.gstart, t.G, psf->kernels, psf->k, kernel,
                                 static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return device_fail(e, "effective_psf");
    return FCAT_OK;
}

static fcat_status slit_geom(double pitch, double width, double tilt_deg, int n_rows, int n_cols, int oversample,
                             SlitGeom &sg)
{
    if (!finite_pos(pitch)) return fail(FCAT_E_INVALID_ARG, "pitch must be finite and > 0");
    if (!(width >= 0.0) || !std::isfinite(width)) return fail(FCAT_E_INVALID_ARG, "width must be finite and >= 0");
    if (!(tilt_deg > 0.0 && tilt_deg < 90.0)) return fail(FCAT_E_INVALID_ARG, "tilt must be in (0, 90) degrees");
    if (n_rows < 1 || n_cols < 1 || (int64_t)n_rows * n_cols > ((int64_t)1 << 26))
        return fail(FCAT_E_INVALID_ARG, "need 1 <= n_rows, n_cols and n_rows n_cols <= 2^26");
    if (oversample < 1 || oversample > 1024) return fail(FCAT_E_INVALID_ARG, "oversample must be in 1..1024");
    const double t = tilt_deg * 3.141592653589793 / 180.0;
    sg.pitch = pitch;
    sg.width = width;
    sg.cos_t = std::cos(t);
    sg.sin_t = std::sin(t);
    sg.h = pitch / (double)oversample;
    sg.n_rows = n_rows;
    sg.n_cols = n_cols;
    double dmin = 1e300, dmax = -1e300;
    for (int ci = 0; ci < 4; ++ci) {
        const int i = (ci & 1) ? n_rows - 1 : 0, j = (ci & 2) ? n_cols - 1 : 0;
        const double x = ((double)j - (double)(n_cols - 1) / 2.0) * pitch;
        const double y = ((double)i - (double)(n_rows - 1) / 2.0) * pitch;
        const double d = sg.cos_t * x + sg.sin_t * y;
        dmin = std::min(dmin, d);
        dmax = std::max(dmax, d);
    }
    const double bl = std::floor(dmin / sg.h + 0.5), bh = std::floor(dmax / sg.h + 0.5);
    if (bh - bl + 1.0 > 1.0e7) return fail(FCAT_E_INVALID_ARG, "too many LSF bins");
    sg.b_min = (int)bl;
    sg.n_bins = (int)(bh - bl) + 1;
    return FCAT_OK;
}

fcat_status fcat_slit_lsf_range(double pitch_mm, double tilt_deg, int32_t n_rows, int32_t n_cols, int32_t oversample,
                                int32_t *b_min, int32_t *n_bins)
{
    g_last_error.clear();
    SlitGeom sg{};
    fcat_status s;
    if ((s = slit_geom(pitch_mm, 0.0, tilt_deg, n_rows, n_cols, oversample, sg))) return s;
    if (!b_min || !n_bins) return fail(FCAT_E_INVALID_ARG, "b_min and n_bins must not be NULL");
    *b_min = sg.b_min;
    *n_bins = sg.n_bins;
    return FCAT_OK;
}

size_t fcat_slit_mtf_workspace_bytes(int32_t n_rows, int32_t n_cols, int32_t n_bins)
{
    if (n_rows < 1 || n_cols < 1 || n_bins < 1) return 0;
    const size_t img = align_up((size_t)n_rows * n_cols * sizeof(float));
    return 2 * img + align_up((size_t)n_bins * sizeof(double)) + align_up((size_t)n_bins * sizeof(int));
}

fcat_status fcat_slit_mtf(const float *kernel, int32_t k, double pitch_mm, double width_mm, double tilt_deg,
                          int32_t n_rows, int32_t n_cols, int32_t oversample, const double *freqs, int32_t n_freq,
                          double *mtf, double *lsf, int32_t *lsf_count, void *workspace, size_t workspace_bytes,
                          void *stream_)
{
    g_last_error.clear();
    SlitGeom sg{};
    fcat_status s;
    if ((s = slit_geom(pitch_mm, width_mm, tilt_deg, n_rows, n_cols, oversample, sg))) return s;
    if (!kernel || k < 1 || k > FCAT_MAX_PSF || (k % 2) == 0)
        return fail(FCAT_E_INVALID_ARG, "kernel must be given with odd k in 1..%d", FCAT_MAX_PSF);
    if (n_freq < 0 || (n_freq > 0 && (!freqs || !mtf))) return fail(FCAT_E_INVALID_ARG, "freqs and mtf must be given");
    const size_t need = fcat_slit_mtf_workspace_bytes(n_rows, n_cols, sg.n_bins);
    if ((s = check_workspace(workspace, workspace_bytes, need))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const size_t img = align_up((size_t)n_rows * n_cols * sizeof(float));
    float *slit = at<float>(workspace, 0), *blurred = at<float>(workspace, img);
    double *lsf_w = lsf ? lsf : at<double>(workspace, 2 * img);
    int *cnt_w = lsf_count ? lsf_count : at<int>(workspace, 2 * img + align_up((size_t)sg.n_bins * sizeof(double)));
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_OPTICS, stream);
        e = launch_slit_image(sg, slit, stream);
    }
    if (e == hipSuccess) {
        StageTimer tm(FCAT_STAGE_PSF, stream);
        e = launch_psf(slit, 1, 1, n_rows, n_cols, kernel, k, blurred, stream);
    }
    if (e == hipSuccess) {
        StageTimer tm(FCAT_STAGE_OPTICS, stream);
        e = launch_slit_lsf(sg, blurred, lsf_w, cnt_w, stream);
        if (e == hipSuccess && n_freq > 0) e = launch_slit_mtf(sg, lsf_w, cnt_w, freqs, n_freq, mtf, stream);
    }
    if (e != hipSuccess) return device_fail(e, "slit_mtf");
    return FCAT_OK;
}

size_t fcat_richardson_lucy_workspace_bytes(int32_t n, int32_t nv, int32_t nu, int32_t k)
{
    if (n < 1 || nv < 1 || nu < 1 || k < 1) return 0;
    const size_t plane = (size_t)nv * nu;
    return 2 * align_up((size_t)n * plane * sizeof(float)) + align_up(plane * sizeof(float)) +
           align_up((size_t)k * k * sizeof(float));
}

fcat_status fcat_richardson_lucy(const float *images, int32_t n, int32_t nv, int32_t nu, const float *kernel, int32_t k,
                                 int32_t iterations, float *out, void *workspace, size_t workspace_bytes,
                                 void *stream_)
{
    g_last_error.clear();
    fcat_status s;
    if (n < 1 || n > 65535 || nv < 1 || nu < 1) return fail(FCAT_E_INVALID_ARG, "need 1 <= n <= 65535, nv, nu >= 1");
    if ((int64_t)nv * nu >= ((int64_t)1 << 31)) return fail(FCAT_E_INVALID_ARG, "nv * nu must be < 2^31");
    if (!kernel || k < 1 || k > FCAT_MAX_PSF || (k % 2) == 0)
        return fail(FCAT_E_INVALID_ARG, "kernel must be given with odd k in 1..%d", FCAT_MAX_PSF);
    if (iterations < 0) return fail(FCAT_E_INVALID_ARG, "iterations must be >= 0");
    if (!images || !out) return fail(FCAT_E_INVALID_ARG, "images and out must not be NULL");
    const int64_t plane = (int64_t)nv * nu, total = (int64_t)n * plane;
    const char *d0 = reinterpret_cast<const char *>(images), *o0 = reinterpret_cast<const char *>(out);
    if (d0 < o0 + total * 4 && o0 < d0 + total * 4) return fail(FCAT_E_INVALID_ARG, "images and out overlap");
    if ((s = check_workspace(workspace, workspace_bytes, fcat_richardson_lucy_workspace_bytes(n, nv, nu, k)))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const size_t big = align_up((size_t)total * sizeof(float));
    float *c = at<float>(workspace, 0), *t = at<float>(workspace, big);
    float *norm = at<float>(workspace, 2 * big);
    float *kt = at<float>(workspace, 2 * big + align_up((size_t)plane * sizeof(float)));
    hipError_t e = hipMemcpyAsync(out, images, (size_t)total * sizeof(float), hipMemcpyDeviceToDevice, stream);
    {
        StageTimer tm(FCAT_STAGE_OPTICS, stream);
        if (e == hipSuccess) e = launch_flip_kernel(kernel, k, kt, stream);
        if (e == hipSuccess) e = launch_fill_value(c, plane, 1.0f, stream);
    }
    if (e == hipSuccess) {
        StageTimer tm(FCAT_STAGE_PSF, stream);
        e = launch_psf(c, 1, 1, nv, nu, kt, k, norm, stream);
    }
    for (int it = 0; e == hipSuccess && it < iterations; ++it) {
        if (k == 15) {
            // both elementwise steps in the convolutions' epilogues
            StageTimer tm(FCAT_STAGE_PSF, stream);
            e = launch_psf_rl(1, out, n, nv, nu, kernel, k, c, images, nullptr, stream);
            if (e == hipSuccess) e = launch_psf_rl(2, c, n, nv, nu, kt, k, out, nullptr, norm, stream);
            continue;
        }
        {
            StageTimer tm(FCAT_STAGE_PSF, stream);
            e = launch_psf(out, n, 1, nv, nu, kernel, k, c, stream);
        }
        if (e == hipSuccess) {
            StageTimer tm(FCAT_STAGE_OPTICS, stream);
            e = launch_rl_ratio(images, c, total, stream);
        }
        if (e == hipSuccess) {
            StageTimer tm(FCAT_STAGE_PSF, stream);
            e = launch_psf(c, n, 1, nv, nu, kt, k, t, stream);
        }
        if (e == hipSuccess) {
            StageTimer tm(FCAT_STAGE_OPTICS, stream);
            e = launch_rl_update(out, t, norm, plane, total, stream);
        }
    }
    if (e != hipSuccess) return device_fail(e, "richardson_lucy");
    return FCAT_OK;
}

fcat_status fcat_count_scale(const fcat_spectral_t *spectral, double counts_per_pixel, float *scale, void *stream)
{
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_spectral(spectral, false, t))) return s;
    if (!spectral->phi || !spectral->eta) return fail(FCAT_E_INVALID_ARG, "phi and eta must not be NULL");
    if (!scale) return fail(FCAT_E_INVALID_ARG, "scale is NULL");
    if (!(counts_per_pixel > 0.0) || !std::isfinite(counts_per_pixel))
        return fail(FCAT_E_INVALID_ARG, "counts_per_pixel must be finite and > 0");
    if ((s = check_pending())) return s;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PROJ, static_cast<hipStream_t>(stream));
        e = launch_count_scale(spectral->phi, spectral->eta, t.gstart, t.E, t.G, counts_per_pixel, scale,
                               static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return device_fail(e, "count_scale");
    return FCAT_OK;
}

fcat_status fcat_poisson(float *Y, int32_t n_ang, int32_t n_groups, int64_t plane, const float *scale,
                         uint64_t seed, int32_t angle_base, void *stream)
{
    g_last_error.clear();
    if (n_ang < 0 || n_groups < 1 || n_groups > FCAT_MAX_GROUPS || plane < 0 || plane >= ((int64_t)1 << 31))
        return fail(FCAT_E_INVALID_ARG, "need n_ang >= 0, 1 <= n_groups <= %d, 0 <= plane < 2^31", FCAT_MAX_GROUPS);
    if (angle_base < 0) return fail(FCAT_E_INVALID_ARG, "angle_base must be >= 0");
    if ((int64_t)n_ang * plane > 0 && (!Y || !scale)) return fail(FCAT_E_INVALID_ARG, "Y and scale must not be NULL");
    fcat_status s;
    if ((s = check_pending())) return s;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_NOISE, static_cast<hipStream_t>(stream));
        e = launch_poisson(Y, n_ang, n_groups, plane, scale, seed, angle_base, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return device_fail(e, "poisson");
    return FCAT_OK;
}

size_t fcat_flood_workspace_bytes(const fcat_spectral_t *spectral, int32_t nv, int32_t nu)
{
    SpecTables t{};
    if (check_spectral(spectral, false, t) || nv < 1 || nu < 1) return 0;
    fcat_geometry_t g{};
    g.nu = nu;
    g.nv = nv;
    return layout(t, &g, false, 0, nullptr, false, 0, true).fixed;
}

fcat_status fcat_flood_profile(const fcat_spectral_t *spectral, const fcat_psf_t *psf, int32_t nv, int32_t nu,
                               float *flood, void *workspace, size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_spectral(spectral, true, t)) || (s = check_psf(psf))) return s;
    if (nv < 1 || nu < 1) return fail(FCAT_E_INVALID_ARG, "nv and nu must be >= 1");
    if (!flood) return fail(FCAT_E_INVALID_ARG, "flood is NULL");
    fcat_geometry_t g{};
    g.nu = nu;
    g.nv = nv;
    Layout L = layout(t, &g, false, 0, nullptr, false, 0, true);
    if ((s = check_workspace(workspace, workspace_bytes, L.fixed))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((s = prep_tables(spectral, nullptr, t, L, workspace, stream))) return s;
    float *unitk = at<float>(workspace, L.unitk);
    float *yf = at<float>(workspace, L.yflood);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PROJ, stream);
        e = psf ? hipSuccess : launch_fill(unitk, t.G, 1.0f, stream);
        if (e == hipSuccess) e = launch_flood_groups(t.Wg, spectral->flood, (int64_t)nv * nu, t.G, yf, stream);
    }
    if (e == hipSuccess) {
        StageTimer tm(FCAT_STAGE_PSF, stream);
        e = launch_psf(yf, 1, t.G, nv, nu, psf ? psf->kernels : unitk, psf ? psf->k : 1, flood, stream);
    }
    if (e != hipSuccess) return device_fail(e, "flood profile");
    return FCAT_OK;
}

fcat_status fcat_log_projection(const float *out, const float *flood, int32_t n_ang, int64_t plane, float floor,
                                float *proj, void *stream)
{
    g_last_error.clear();
    if (n_ang < 0 || plane < 0) return fail(FCAT_E_INVALID_ARG, "n_ang and plane must be >= 0");
    if (!(floor >= 0.0f) || !std::isfinite(floor)) return fail(FCAT_E_INVALID_ARG, "floor must be finite and >= 0");
    if ((int64_t)n_ang * plane > 0 && (!out || !flood || !proj))
        return fail(FCAT_E_INVALID_ARG, "out, flood and proj must not be NULL");
    fcat_status s;
    if ((s = check_pending())) return s;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PROJ, static_cast<hipStream_t>(stream));
        e = launch_log_projection(out, flood, n_ang, plane, floor, proj, static_cast<hipStream_t>(stream));
    }
    if (e != hipSuccess) return device_fail(e, "log_projection");
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
    int8_t *labels_bm = labels_bm_at(bricks, phantom);
    G.bricks = bricks;
    G.labels_bm = labels_bm;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_PREP, stream);
        G.clip = clip_at(bricks, phantom);
        e = launch_build_bricks(phantom->labels, phantom->nx, phantom->ny, phantom->nz, bricks, labels_bm,
                                clip_at(bricks, phantom), stream);
    }
    if (e != hipSuccess) return device_fail(e, "build_bricks");
    {
        StageTimer tm(FCAT_STAGE_TRACE, stream);
        e = launch_pathlengths(G, phantom->labels, n_mat, a_begin, a_end - a_begin, L, stream);
    }
    if (e != hipSuccess) return device_fail(e, "pathlengths");
    return FCAT_OK;
}

fcat_status fcat_walk_stats(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom, int32_t a_begin,
                            int32_t a_end, int64_t *counts, void *workspace, size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    fcat_status s;
    if ((s = check_geometry(geometry)) || (s = check_phantom(phantom))) return s;
    if (a_begin < 0 || a_end > geometry->n_angles || a_begin >= a_end)
        return fail(FCAT_E_INVALID_ARG, "need 0 <= a_begin < a_end <= n_angles");
    if (!counts) return fail(FCAT_E_INVALID_ARG, "counts is NULL");
    if ((s = check_workspace(workspace, workspace_bytes, align_up(brick_bytes(phantom))))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    TraceGeom G = make_geom(geometry, phantom);
    int8_t *bricks = static_cast<int8_t *>(workspace);
    G.bricks = bricks;
    G.labels_bm = labels_bm_at(bricks, phantom);
    hipError_t e = launch_zero_ints(reinterpret_cast<int *>(counts), 2 * kWalkCounts, stream);
    int *clip = clip_at(bricks, phantom);
    G.clip = clip;
    if (e == hipSuccess)
        e = launch_build_bricks(phantom->labels, phantom->nx, phantom->ny, phantom->nz, bricks,
                                const_cast<int8_t *>(G.labels_bm), clip, stream);
    if (e == hipSuccess)
        e = launch_walk_stats(G, a_begin, a_end - a_begin, reinterpret_cast<unsigned long long *>(counts), stream);
    if (e != hipSuccess) return device_fail(e, "walk_stats");
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

// Eq. 3 on given path lengths, its tables in `workspace` (the caller's, or
// this device's copy of the static scratch).  scratch_ws makes the workspace
// the static scratch, looked up only once the arguments have been checked.
static fcat_status spectral_impl(const float *Lin, int64_t n, const fcat_spectral_t *spectral, const float *i0,
                                 const float *S, const float *s_bin, fcat_mode mode, float *Y, void *workspace,
                                 size_t workspace_bytes, bool scratch_ws, void *stream_)
{
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
    if (scratch_ws) {
        if (L.fixed > kStaticScratchBytes)
            return fail(FCAT_E_UNSUPPORTED, "the tables need %zu bytes, the static scratch holds %zu", L.fixed,
                        kStaticScratchBytes);
        if (n == 0) return FCAT_OK;
        if ((s = static_scratch(&workspace))) return s;
        workspace_bytes = kStaticScratchBytes;
    }
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

fcat_status fcat_spectral(const float *Lin, int64_t n, const fcat_spectral_t *spectral, const float *i0,
                          const float *S, const float *s_bin, fcat_mode mode, float *Y, void *workspace,
                          size_t workspace_bytes, void *stream)
{
    g_last_error.clear();
    return spectral_impl(Lin, n, spectral, i0, S, s_bin, mode, Y, workspace, workspace_bytes, false, stream);
}

fcat_status fcat_spectral_static(const float *Lin, int64_t n, const fcat_spectral_t *spectral, const float *i0,
                                 const float *S, const float *s_bin, fcat_mode mode, float *Y, void *stream)
{
    g_last_error.clear();
    return spectral_impl(Lin, n, spectral, i0, S, s_bin, mode, Y, nullptr, 0, true, stream);
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

int32_t fcat_mlp_param_count(int32_t n_in, int32_t n_out)
{
    if (n_in < 1 || n_in > FCAT_MLP_MAX_IO || n_out < 1 || n_out > FCAT_MLP_MAX_IO) return 0;
    return mlp_param_count(n_in, n_out);
}

size_t fcat_mlp_workspace_bytes(const fcat_spectral_t *spectral, int64_t batch)
{
    SpecTables t{};
    if (check_spectral(spectral, false, t) || batch < 1 || batch > FCAT_MLP_MAX_BATCH) return 0;
    return mlp_layout(t, batch).total;
}

fcat_status fcat_mlp_linear_term(const fcat_spectral_t *spectral, float *lin, void *workspace, size_t workspace_bytes,
                                 void *stream_)
{
    g_last_error.clear();
    SpecTables t{};
    fcat_status s;
    if ((s = check_spectral(spectral, true, t))) return s;
    if (!lin) return fail(FCAT_E_INVALID_ARG, "lin is NULL");
    Layout L = layout(t, nullptr, false);
    if ((s = check_workspace(workspace, workspace_bytes, L.fixed))) return s;
    if ((s = check_pending())) return s;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if ((s = prep_tables(spectral, nullptr, t, L, workspace, stream))) return s;
    hipError_t e = launch_mlp_linear(spectral->mu, t, lin, stream);
    if (e != hipSuccess) return device_fail(e, "mlp_linear");
    return FCAT_OK;
}

// Shared set-up of the fcat_mlp_* calls.
static fcat_status mlp_begin(const fcat_surrogate_t *u, const fcat_spectral_t *spectral, const float *params,
                             int64_t batch, void *workspace, size_t workspace_bytes, hipStream_t stream, SpecTables &t,
                             MlpLayout &ml, MlpTables &mt)
{
    fcat_status s;
    if ((s = check_spectral(spectral, true, t))) return s;
    if ((s = check_surrogate(u, t, false))) return s;
    if (!params) return fail(FCAT_E_INVALID_ARG, "params is NULL");
    ml = mlp_layout(t, batch);
    if ((s = check_workspace(workspace, workspace_bytes, ml.total))) return s;
    if ((s = check_pending())) return s;
    if ((s = prep_tables(spectral, nullptr, t, ml.base, workspace, stream))) return s;
    return prep_mlp(u, params, t, ml.base, workspace, stream, mt);
}

fcat_status fcat_mlp_forward(const fcat_surrogate_t *surrogate, const fcat_spectral_t *spectral, const float *L,
                             int64_t n, float *Yprim, void *workspace, size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    if (n < 0) return fail(FCAT_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!L || !Yprim)) return fail(FCAT_E_INVALID_ARG, "L and Yprim must not be NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SpecTables t{};
    MlpLayout ml{};
    MlpTables mt{};
    fcat_status s;
    if ((s = mlp_begin(surrogate, spectral, surrogate ? surrogate->params : nullptr, 1, workspace, workspace_bytes,
                       stream, t, ml, mt)))
        return s;
    if (n == 0) return FCAT_OK;
    SurrogateIO io{};
    io.L = L;
    io.n = n;
    io.plane = n;
    io.Y = Yprim;
    io.force_mlp = 1;
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_MLP, stream);
        e = launch_mlp_spectral(t, mt, io, stream);
    }
    if (e != hipSuccess) return device_fail(e, "mlp_forward");
    return FCAT_OK;
}

fcat_status fcat_mlp_gradients(const fcat_surrogate_t *surrogate, const fcat_spectral_t *spectral, const float *L,
                               const float *Yprim, int64_t n, float *grad, float *loss, void *workspace,
                               size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    if (n < 1 || n > FCAT_MLP_MAX_BATCH) return fail(FCAT_E_INVALID_ARG, "n must be in 1..%d", FCAT_MLP_MAX_BATCH);
    if (!L || !Yprim || !grad) return fail(FCAT_E_INVALID_ARG, "L, Yprim and grad must not be NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SpecTables t{};
    MlpLayout ml{};
    MlpTables mt{};
    fcat_status s;
    if ((s = mlp_begin(surrogate, spectral, surrogate ? surrogate->params : nullptr, n, workspace, workspace_bytes,
                       stream, t, ml, mt)))
        return s;
    float *partial = at<float>(workspace, ml.partial);
    float *lp = at<float>(workspace, ml.loss_partial);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_MLP, stream);
        e = launch_mlp_grad(t, mt, L, Yprim, n, nullptr, 0, (int)n, partial, lp, stream);
        if (e == hipSuccess)
            e = launch_mlp_reduce_adam(partial, (int)((n + kWave - 1) / kWave), ml.P, grad, nullptr, nullptr, nullptr,
                                       0, 0.f, 0.f, 0.f, 0.f, lp, 1.0f / ((float)n * (float)t.G), loss, stream);
    }
    if (e != hipSuccess) return device_fail(e, "mlp_gradients");
    return FCAT_OK;
}

static fcat_status check_train(const fcat_mlp_train_t *tr)
{
    if (!tr) return fail(FCAT_E_INVALID_ARG, "train is NULL");
    if (!tr->params || !tr->adam_m || !tr->adam_v)
        return fail(FCAT_E_INVALID_ARG, "train params and Adam moments must not be NULL");
    if (tr->step < 0) return fail(FCAT_E_INVALID_ARG, "train step must be >= 0");
    if (!(tr->lr > 0.0f) || !(tr->beta1 >= 0.0f && tr->beta1 < 1.0f) || !(tr->beta2 >= 0.0f && tr->beta2 < 1.0f) ||
        !(tr->eps >= 0.0f))
        return fail(FCAT_E_INVALID_ARG, "Adam hyper-parameters out of range");
    return FCAT_OK;
}

static hipError_t train_one(fcat_mlp_train_t *train, const SpecTables &t, MlpTables &mt, const MlpLayout &ml,
                            void *workspace, const float *L, const float *Yprim, int64_t n, const int32_t *order,
                            int64_t base, int count, float *loss, hipStream_t stream)
{
    float *partial = at<float>(workspace, ml.partial);
    float *lp = at<float>(workspace, ml.loss_partial);
    StageTimer tm(FCAT_STAGE_MLP, stream);
    hipError_t e = launch_mlp_grad(t, mt, L, Yprim, n, order, base, count, partial, lp, stream);
    if (e == hipSuccess)
        e = launch_mlp_reduce_adam(partial, (count + kWave - 1) / kWave, ml.P, nullptr, train->params, train->adam_m,
                                   train->adam_v, train->step + 1, train->lr, train->beta1, train->beta2, train->eps,
                                   lp, 1.0f / ((float)count * (float)t.G), loss, stream, at<int>(workspace, ml.fcnt),
                                   at<uint32_t>(workspace, ml.finv), const_cast<uint4 *>(mt.frag));
    if (e == hipSuccess) train->step += 1;
    return e;
}

// Before the first train_one of a call: mlp_begin has built the fragment
// views of the current parameters; each Adam step then rewrites the
// training views of the parameters it updates, through the table of
// fragment elements per parameter built here.
static hipError_t train_begin(const SpecTables &t, const MlpLayout &ml, void *workspace, hipStream_t stream)
{
    StageTimer tm(FCAT_STAGE_MLP, stream);
    return launch_mlp_frag_inverse(t.M, t.G, at<int>(workspace, ml.fcnt), at<uint32_t>(workspace, ml.finv), stream);
}

fcat_status fcat_mlp_train_step(fcat_mlp_train_t *train, const fcat_surrogate_t *surrogate,
                                const fcat_spectral_t *spectral, const float *L, const float *Yprim, int64_t n,
                                const int32_t *order, int64_t base, int32_t count, float *loss, void *workspace,
                                size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    fcat_status s;
    if ((s = check_train(train))) return s;
    if (count < 1 || count > FCAT_MLP_MAX_BATCH) return fail(FCAT_E_INVALID_ARG, "count must be in 1..%d", FCAT_MLP_MAX_BATCH);
    if (!L || !Yprim || n < 1 || base < 0 || (!order && base + count > n))
        return fail(FCAT_E_INVALID_ARG, "bad sample range");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SpecTables t{};
    MlpLayout ml{};
    MlpTables mt{};
    if ((s = mlp_begin(surrogate, spectral, train->params, count, workspace, workspace_bytes, stream, t, ml, mt)))
        return s;
    hipError_t e = train_begin(t, ml, workspace, stream);
    if (e == hipSuccess) e = train_one(train, t, mt, ml, workspace, L, Yprim, n, order, base, count, loss, stream);
    if (e != hipSuccess) return device_fail(e, "mlp_train_step");
    return FCAT_OK;
}

fcat_status fcat_mlp_train_epoch(fcat_mlp_train_t *train, const fcat_surrogate_t *surrogate,
                                 const fcat_spectral_t *spectral, const float *L, const float *Yprim, int64_t n,
                                 const int32_t *order, int32_t batch, float *batch_loss, void *workspace,
                                 size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    fcat_status s;
    if ((s = check_train(train))) return s;
    if (batch < 1 || batch > FCAT_MLP_MAX_BATCH) return fail(FCAT_E_INVALID_ARG, "batch must be in 1..%d", FCAT_MLP_MAX_BATCH);
    if (!L || !Yprim || n < 1) return fail(FCAT_E_INVALID_ARG, "bad sample range");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SpecTables t{};
    MlpLayout ml{};
    MlpTables mt{};
    if ((s = mlp_begin(surrogate, spectral, train->params, batch, workspace, workspace_bytes, stream, t, ml, mt)))
        return s;
    hipError_t e0 = train_begin(t, ml, workspace, stream);
    if (e0 != hipSuccess) return device_fail(e0, "mlp_train_epoch");
    int64_t b = 0;
    for (int64_t base = 0; base < n; base += batch, ++b) {
        const int count = (int)std::min<int64_t>(batch, n - base);
        hipError_t e = train_one(train, t, mt, ml, workspace, L, Yprim, n, order, base, count,
                                 batch_loss ? batch_loss + b : nullptr, stream);
        if (e != hipSuccess) return device_fail(e, "mlp_train_epoch");
    }
    return FCAT_OK;
}

fcat_status fcat_mlp_validate(const fcat_surrogate_t *surrogate, const fcat_spectral_t *spectral, const float *L,
                              const float *Yprim, int64_t n, float threshold, int32_t min_count, float *cell_err,
                              uint8_t *cell_ok, int32_t *cell_count, void *workspace, size_t workspace_bytes,
                              void *stream_)
{
    g_last_error.clear();
    if (n < 1 || !L || !Yprim || !cell_ok) return fail(FCAT_E_INVALID_ARG, "L, Yprim, cell_ok and n >= 1 are needed");
    if (!(threshold >= 0.0f) || min_count < 1) return fail(FCAT_E_INVALID_ARG, "threshold >= 0 and min_count >= 1");
    if (!surrogate || !std::isfinite(surrogate->cell_lo) || !std::isfinite(surrogate->cell_hi) ||
        !(surrogate->cell_lo < surrogate->cell_hi))
        return fail(FCAT_E_INVALID_ARG, "surrogate cell range must be finite with cell_lo < cell_hi");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SpecTables t{};
    MlpLayout ml{};
    MlpTables mt{};
    fcat_status s;
    if ((s = mlp_begin(surrogate, spectral, surrogate->params, 1, workspace, workspace_bytes, stream, t, ml, mt)))
        return s;
    const int ncell = t.M * FCAT_MLP_CELLS;
    unsigned *bits = at<unsigned>(workspace, ml.cells);
    int *count = reinterpret_cast<int *>(bits + FCAT_MLP_MAX_IO * FCAT_MLP_CELLS);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_MLP, stream);
        e = launch_zero_ints(reinterpret_cast<int *>(bits), 2 * FCAT_MLP_MAX_IO * FCAT_MLP_CELLS, stream);
        if (e == hipSuccess) e = launch_mlp_validate(t, mt, L, Yprim, n, bits, count, stream);
        if (e == hipSuccess) e = launch_mlp_cells(bits, count, ncell, threshold, min_count, cell_err, cell_ok, stream);
        if (e == hipSuccess && cell_count)
            e = hipMemcpyAsync(cell_count, count, (size_t)ncell * sizeof(int), hipMemcpyDeviceToDevice, stream);
    }
    if (e != hipSuccess) return device_fail(e, "mlp_validate");
    return FCAT_OK;
}

fcat_status fcat_mlp_setup(const fcat_spectral_t *spectral, const float *lin, const float *L, const float *Yprim,
                           int64_t n, float *in_scale, float *out_scale, float *tau_max, void *workspace,
                           size_t workspace_bytes, void *stream_)
{
    g_last_error.clear();
    if (n < 1 || !lin || !L || !Yprim || !in_scale || !out_scale || !tau_max)
        return fail(FCAT_E_INVALID_ARG, "lin, L, Yprim, in_scale, out_scale, tau_max and n >= 1 are needed");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SpecTables t{};
    fcat_status s;
    if ((s = check_spectral(spectral, true, t))) return s;
    if (t.M > FCAT_MLP_MAX_IO || t.G > FCAT_MLP_MAX_IO)
        return fail(FCAT_E_INVALID_ARG, "n_mat and n_groups must be <= %d", FCAT_MLP_MAX_IO);
    const MlpLayout ml = mlp_layout(t, 1);
    if ((s = check_workspace(workspace, workspace_bytes, ml.total))) return s;
    if ((s = check_pending())) return s;
    if ((s = prep_tables(spectral, nullptr, t, ml.base, workspace, stream))) return s;
    float *mbar = at<float>(workspace, ml.base.mbar);
    float *partial = at<float>(workspace, ml.stats);
    hipError_t e;
    {
        StageTimer tm(FCAT_STAGE_MLP, stream);
        e = launch_mlp_mbar(t, lin, mbar, stream);
        if (e == hipSuccess)
            e = launch_mlp_stats(t, lin, mbar, L, Yprim, n, partial, in_scale, out_scale, tau_max, stream);
    }
    if (e != hipSuccess) return device_fail(e, "mlp_setup");
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
