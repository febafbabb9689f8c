// gfx950 kernels of the polyenergetic cone-beam projector.
//
// One lane follows one ray (one detector pixel of one angle); one wavefront
// covers 64 consecutive detector columns of one row, so its rays are
// neighbours in space (they share voxel cache lines), have nearly equal
// lengths (little divergence) and write their results with coalesced stores.
//
// Ray traversal (Sec. II.F: a projection is the line integral of the
// attenuation along the ray; Sec. II.C: the phantom holds material labels,
// so the integral is sum_m mu_m(E) L_m): entry and exit are found in FP64 by
// the slab method, the ray is re-based at its entry point and then walked
// in FP32 distance from there (incremental form of Siddon's exact method),
// over bricks of voxels first and over single voxels only inside bricks
// whose labels differ.  Each plane crossing is t0 + k dt evaluated with one
// rounding, so the error does not grow with the number of planes.  Path
// length is charged to a material only when the label changes, with
// compensated (Kahan) summation, so its error scales with the number of
// material transitions rather than with the number of voxels.
#include "fcat_internal.h"

#include <cmath>

namespace fcat {
namespace {

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Hardware hands consecutive workgroups to the 8 XCDs in turn.  Remap so that
// each XCD (and its L2) works through one contiguous range of rays.  The
// grid is padded to a multiple of kXcds so the map is a bijection.
__device__ __forceinline__ int xcd_block(int nblk_padded)
{
    const int b = blockIdx.x;
    const int per = nblk_padded / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Per-ray constants of the two-level walk.  Distances t are measured in mm
// from the point where the ray enters the grid.
struct Ray {
    float t_end;        // exit distance
    float t0[3];        // first voxel-plane crossing per axis (inf if parallel)
    float dt[3];        // distance between voxel-plane crossings
    float inv_dt[3];    // 1 / dt (0 if parallel)
    float tc0[3];       // first brick-plane crossing per axis (inf if parallel)
    float dtc[3];       // distance between brick-plane crossings
    int i0[3];          // entry voxel
    int sgn[3];         // direction of travel per axis: +1, -1, or 0 if parallel
};

// FP64 set-up of the ray from the source to the centre of pixel (iv, iu):
// entry and exit by the slab method, then everything re-based at the entry
// point and rounded once to FP32.
__device__ __forceinline__ bool setup_ray(const TraceGeom &G, double ct, double st, int iv, int iu, Ray &r)
{
    const double pu = ((double)iu - G.cu) * G.du + G.off_u;
    const double pv = ((double)iv - G.cv) * G.dv + G.off_v;
    const double s[3] = {G.sid * ct, G.sid * st, 0.0};
    const double p[3] = {-G.back * ct - pu * st, -G.back * st + pu * ct, pv};
    double d[3], inv[3];
    double amin = 0.0, amax = 1.0;
    bool inside = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        d[ax] = p[ax] - s[ax];
        const double lo = G.lo[ax];
        const double hi = G.lo[ax] + G.n[ax] * G.h[ax];
        if (d[ax] == 0.0) {
            inv[ax] = 0.0;
            inside = inside && s[ax] >= lo && s[ax] < hi;
        } else {
            inv[ax] = 1.0 / d[ax];
            const double a0 = (lo - s[ax]) * inv[ax];
            const double a1 = (hi - s[ax]) * inv[ax];
            amin = fmax(amin, fmin(a0, a1));
            amax = fmin(amax, fmax(a0, a1));
        }
    }
    if (!inside || !(amax > amin)) return false;
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    r.t_end = (float)((amax - amin) * len);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double q = (s[ax] + amin * d[ax] - G.lo[ax]) * G.inv_h[ax];
        // entering through a plane: the voxel beyond it in the direction of travel
        int i = d[ax] < 0.0 ? (int)ceil(q) - 1 : (int)floor(q);
        i = min(max(i, 0), G.n[ax] - 1);
        r.i0[ax] = i;
        if (d[ax] != 0.0) {
            const int plane = d[ax] > 0.0 ? i + 1 : i;
            const double ap = (G.lo[ax] + plane * G.h[ax] - s[ax]) * inv[ax];
            const double step = G.h[ax] * len * fabs(inv[ax]);
            r.t0[ax] = (float)fmax((ap - amin) * len, 0.0);
            r.dt[ax] = (float)step;
            r.inv_dt[ax] = (float)(1.0 / step);
            const int b = i / G.B;
            const int bplane = (d[ax] > 0.0 ? b + 1 : b) * G.B;
            const double bp = (G.lo[ax] + bplane * G.h[ax] - s[ax]) * inv[ax];
            r.tc0[ax] = (float)fmax((bp - amin) * len, 0.0);
            r.dtc[ax] = (float)(step * G.B);
            r.sgn[ax] = d[ax] > 0.0 ? 1 : -1;
        } else {
            r.t0[ax] = INFINITY;
            r.dt[ax] = 0.0f;
            r.inv_dt[ax] = 0.0f;
            r.tc0[ax] = INFINITY;
            r.dtc[ax] = 0.0f;
            r.sgn[ax] = 0;
        }
    }
    return true;
}

// Compensated add of x to material m (compare-select over the padded
// material count, so the register arrays are never indexed dynamically).
// Labels outside 0..MP-1 match nothing and add nothing.
template <int MP>
__device__ __forceinline__ void kahan_add(float (&L)[MP], float (&C)[MP], int m, float x)
{
    float l = 0.0f, c = 0.0f;
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        l = (k == m) ? L[k] : l;
        c = (k == m) ? C[k] : c;
    }
    const float y = x - c;
    const float t = l + y;
    c = (t - l) - y;
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        L[k] = (k == m) ? t : L[k];
        C[k] = (k == m) ? c : C[k];
    }
}

// Number of crossings of one axis at or before distance T: the k with
// t0 + (k-1) dt <= T < t0 + k dt, evaluated with the same rounded formula
// the walk uses, so that a walk resumed at T stays consistent with one that
// had stepped through every plane.
__device__ __forceinline__ float crossings_before(float T, float t0, float dt, float inv_dt)
{
    if (!(T >= t0)) return 0.0f;
    float k = floorf((T - t0) * inv_dt) + 1.0f;
    if (k > 0.0f && fmaf(k - 1.0f, dt, t0) > T) k -= 1.0f;
    if (fmaf(k, dt, t0) <= T) k += 1.0f;
    return k;
}

// Two-level exact walk (Siddon's path lengths, found hierarchically).
//
// The grid is tiled into B x B x B bricks; bricks[] holds the label of a
// brick whose voxels all share one label, or -1.  The coarse walk crosses
// brick planes; a uniform brick contributes its whole segment to its label
// in one step, and only inside mixed bricks does the fine walk cross the
// individual voxel planes.  Crossing k + 1 of an axis lies at t0 + k dt (one
// rounding from its exact value) for both levels; path length is charged to
// a material only when the label changes, with compensated summation.
template <int MP>
__device__ __forceinline__ void trace_bricks(const Ray &r, bool hit, const TraceGeom &G,
                                             const int8_t *__restrict__ labels,
                                             const int8_t *__restrict__ bricks, float (&L)[MP])
{
    float C[MP];
#pragma unroll
    for (int m = 0; m < MP; ++m) {
        L[m] = 0.0f;
        C[m] = 0.0f;
    }
    if (!hit) return;
    const float t_end = r.t_end;
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const int nbx = G.nb[0], nby = G.nb[1];
    const int last_vox = nx * ny * nz - 1;
    const int last_brick = G.nb[0] * G.nb[1] * G.nb[2] - 1;
    const int vstride[3] = {1, nx, nx * ny};
    const int bstride[3] = {1, nbx, nbx * nby};

    float kc[3] = {0.0f, 0.0f, 0.0f};
    float tc[3] = {r.tc0[0], r.tc0[1], r.tc0[2]};
    const int db[3] = {r.sgn[0] * bstride[0], r.sgn[1] * bstride[1], r.sgn[2] * bstride[2]};
    const int dv[3] = {r.sgn[0] * vstride[0], r.sgn[1] * vstride[1], r.sgn[2] * vstride[2]};
    int blin = (r.i0[2] / G.B * nby + r.i0[1] / G.B) * nbx + r.i0[0] / G.B;
    int bl = bricks[blin];
    int cur = -1;
    float run = 0.0f;
    float T_in = 0.0f;
    int budget = G.nb[0] + G.nb[1] + G.nb[2] + 4;
    bool active = true;
    while (active) {
        const float tco = fminf(tc[0], fminf(tc[1], tc[2]));
        const bool last = !(tco < t_end) || --budget < 0;
        const float T_out = last ? t_end : tco;
        if (bl >= 0) {
            if (bl != cur) {
                kahan_add<MP>(L, C, cur, T_in - run);
                cur = bl;
                run = T_in;
            }
        } else {
            // fine walk over [T_in, T_out): resume the voxel counters at T_in
            float k[3], t[3];
            int lin = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                k[a] = r.sgn[a] ? crossings_before(T_in, r.t0[a], r.dt[a], r.inv_dt[a]) : 0.0f;
                t[a] = r.sgn[a] ? fmaf(k[a], r.dt[a], r.t0[a]) : INFINITY;
                const int ia = min(max(r.i0[a] + r.sgn[a] * (int)k[a], 0), G.n[a] - 1);
                lin += ia * vstride[a];
            }
            int lab = labels[lin];
            if (lab != cur) {
                kahan_add<MP>(L, C, cur, T_in - run);
                cur = lab;
                run = T_in;
            }
            for (int f = 0; f < 3 * G.B + 3; ++f) {
                const float tn = fminf(t[0], fminf(t[1], t[2]));
                if (!(tn < T_out)) break;
                const bool bx = (t[0] == tn);
                const bool by = !bx && (t[1] == tn);
                const bool bz = !bx && !by;
                lin += (bx ? dv[0] : 0) + (by ? dv[1] : 0) + (bz ? dv[2] : 0);
                k[0] += bx ? 1.0f : 0.0f;
                k[1] += by ? 1.0f : 0.0f;
                k[2] += bz ? 1.0f : 0.0f;
                t[0] = r.sgn[0] ? fmaf(k[0], r.dt[0], r.t0[0]) : INFINITY;
                t[1] = r.sgn[1] ? fmaf(k[1], r.dt[1], r.t0[1]) : INFINITY;
                t[2] = r.sgn[2] ? fmaf(k[2], r.dt[2], r.t0[2]) : INFINITY;
                lab = labels[min(max(lin, 0), last_vox)];
                if (lab != cur) {
                    kahan_add<MP>(L, C, cur, tn - run);
                    cur = lab;
                    run = tn;
                }
            }
        }
        if (last) {
            active = false;
        } else {
            const bool bx = (tc[0] == tco);
            const bool by = !bx && (tc[1] == tco);
            const bool bz = !bx && !by;
            blin += (bx ? db[0] : 0) + (by ? db[1] : 0) + (bz ? db[2] : 0);
            kc[0] += bx ? 1.0f : 0.0f;
            kc[1] += by ? 1.0f : 0.0f;
            kc[2] += bz ? 1.0f : 0.0f;
            tc[0] = r.sgn[0] ? fmaf(kc[0], r.dtc[0], r.tc0[0]) : INFINITY;
            tc[1] = r.sgn[1] ? fmaf(kc[1], r.dtc[1], r.tc0[1]) : INFINITY;
            tc[2] = r.sgn[2] ? fmaf(kc[2], r.dtc[2], r.tc0[2]) : INFINITY;
            T_in = tco;
            bl = bricks[min(max(blin, 0), last_brick)];
        }
    }
    kahan_add<MP>(L, C, cur, t_end - run);
}

// sum over the bins of one group of w_e exp(-sum_m mu[e][m] L_m)   (Eq. 3)
template <int MP>
__device__ __forceinline__ float group_sum(const float (&L)[MP], const SpecTables &T, int e0, int e1)
{
    float acc = 0.0f;
    for (int e = e0; e < e1; ++e) {
        const float *mrow = T.muT + e * MP;
        float P = 0.0f;
#pragma unroll
        for (int m = 0; m < MP; ++m) P = fmaf(mrow[m], L[m], P);
        acc = fmaf(T.w[e], expf(-P), acc);
    }
    return acc;
}

__device__ __forceinline__ double angle_of(const TraceGeom &G, int a)
{
    return G.angles ? G.angles[a] : (2.0 * M_PI) * (double)a / (double)G.n_angles;
}

// ------------------------------------------------------------ projector

template <int MP>
__global__ __launch_bounds__(kBlock) void k_project_rows(TraceGeom G, const int8_t *__restrict__ labels,
                                                         SpecTables T, const float *__restrict__ flood,
                                                         const float *__restrict__ scatter, int a0,
                                                         int n_ang, int waves_per_row, int nblk_pad,
                                                         float *__restrict__ Y, float *__restrict__ out)
{
    const int blk = xcd_block(nblk_pad);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blk * (kBlock / kWave) + wave;
    if (gw >= n_ang * G.nv * waves_per_row) return;
    const int row = gw / waves_per_row;
    const int iu = (gw - row * waves_per_row) * kWave + lane;
    const int al = row / G.nv;
    const int iv = row - al * G.nv;
    const int a = a0 + al;
    const bool valid = iu < G.nu;

    double st, ct;
    sincos(angle_of(G, a), &st, &ct);
    float L[MP];
    Ray r{};
    const bool hit = valid && setup_ray(G, ct, st, iv, iu, r);
    trace_bricks<MP>(r, hit, G, labels, G.bricks, L);
    const bool any_hit = __ballot(hit) != 0;
    if (!valid) return;

    const int64_t plane = (int64_t)G.nu * G.nv;
    const int64_t pix = (int64_t)iv * G.nu + iu;
    const float i0 = flood ? flood[pix] : 1.0f;
    const float sc = scatter ? scatter[(int64_t)a * plane + pix] : 0.0f;
    float total = 0.0f;
    for (int g = 0; g < T.G; ++g) {
        const float acc = any_hit ? group_sum<MP>(L, T, T.gstart[g], T.gstart[g + 1]) : T.Wg[g];
        const float y = fmaf(i0, acc, T.Wsg[g] * sc);
        if (Y)
            Y[((int64_t)al * T.G + g) * plane + pix] = y;
        else
            total += y;
    }
    if (!Y) out[(int64_t)a * plane + pix] = total;
}

template <int MP>
__global__ __launch_bounds__(kBlock) void k_pathlengths(TraceGeom G, const int8_t *__restrict__ labels,
                                                        int n_mat, int a0, int n_ang, int waves_per_row,
                                                        int nblk_pad, float *__restrict__ Lout)
{
    const int blk = xcd_block(nblk_pad);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blk * (kBlock / kWave) + wave;
    if (gw >= n_ang * G.nv * waves_per_row) return;
    const int row = gw / waves_per_row;
    const int iu = (gw - row * waves_per_row) * kWave + lane;
    const int al = row / G.nv;
    const int iv = row - al * G.nv;
    if (iu >= G.nu) return;
    double st, ct;
    sincos(angle_of(G, a0 + al), &st, &ct);
    float L[MP];
    Ray r{};
    const bool hit = setup_ray(G, ct, st, iv, iu, r);
    trace_bricks<MP>(r, hit, G, labels, G.bricks, L);
    float *dst = Lout + (((int64_t)al * G.nv + iv) * G.nu + iu) * n_mat;
#pragma unroll
    for (int m = 0; m < MP; ++m)
        if (m < n_mat) dst[m] = L[m];
}

template <int MP>
__global__ __launch_bounds__(kBlock) void k_spectral(const float *__restrict__ Lin, int64_t n, SpecTables T,
                                                     const float *__restrict__ i0,
                                                     const float *__restrict__ S, float *__restrict__ Y)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    float L[MP];
#pragma unroll
    for (int m = 0; m < MP; ++m) L[m] = m < T.M ? Lin[r * T.M + m] : 0.0f;
    const float f = i0 ? i0[r] : 1.0f;
    const float sc = S ? S[r] : 0.0f;
    for (int g = 0; g < T.G; ++g) {
        const float acc = group_sum<MP>(L, T, T.gstart[g], T.gstart[g + 1]);
        Y[(int64_t)g * n + r] = fmaf(f, acc, T.Wsg[g] * sc);
    }
}

// ------------------------------------------------------- tables and checks

__global__ __launch_bounds__(kBlock) void k_prep_tables(const float *__restrict__ mu,
                                                        const float *__restrict__ phi,
                                                        const float *__restrict__ eta,
                                                        const float *__restrict__ s_bin, SpecTables T,
                                                        float *__restrict__ muT, float *__restrict__ w,
                                                        float *__restrict__ Wg, float *__restrict__ Wsg)
{
    for (int e = threadIdx.x; e < T.E; e += kBlock) {
        w[e] = phi[e] * eta[e];
        for (int m = 0; m < T.mp; ++m) muT[e * T.mp + m] = m < T.M ? mu[(int64_t)m * T.E + e] : 0.0f;
    }
    const int g = threadIdx.x;
    if (g < T.G) {
        double a = 0.0, b = 0.0;
        for (int e = T.gstart[g]; e < T.gstart[g + 1]; ++e) {
            const double we = (double)(phi[e] * eta[e]);
            a += we;
            b += we * (s_bin ? (double)s_bin[e] : 1.0);
        }
        Wg[g] = (float)a;
        Wsg[g] = (float)b;
    }
}

__global__ __launch_bounds__(kBlock) void k_check_labels(const int8_t *__restrict__ lab, int64_t n,
                                                         int n_mat, int *flag)
{
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int v = lab[i];
        bad |= (v < 0 || v >= n_mat);
    }
    if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const float *__restrict__ x, int64_t n, int *flag)
{
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        bad |= !isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

__global__ void k_zero_ints(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------- PSF
//
// out[a][v][u] = sum_g sum_{i,j} K_g[k-1-i][k-1-j] T_g[v + i][u + j], the
// true convolution written as a correlation with the flipped kernel over an
// LDS tile T_g whose origin is (v0 - c, u0 - c) and which is zero outside
// the detector.  A workgroup owns 64 columns x 4*ROWS rows; each lane owns
// one column and ROWS consecutive rows, so every LDS value it reads feeds up
// to ROWS outputs.  Kernel weights are wave-uniform (scalar loads).

template <int K, int ROWS>
__global__ __launch_bounds__(kBlock) void k_psf(const float *__restrict__ Y, int G, int nv, int nu,
                                                const float *__restrict__ ker, float *__restrict__ out)
{
    constexpr int C = (K - 1) / 2;
    constexpr int TU = kWave;
    constexpr int TV = (kBlock / kWave) * ROWS;
    constexpr int LW = TU + K - 1;
    constexpr int LH = TV + K - 1;
    __shared__ float tile[LH * LW];
    const int u0 = blockIdx.x * TU;
    const int v0 = blockIdx.y * TV;
    const int a = blockIdx.z;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t plane = (int64_t)nv * nu;
    float acc[ROWS];
#pragma unroll
    for (int o = 0; o < ROWS; ++o) acc[o] = 0.0f;

    for (int g = 0; g < G; ++g) {
        const float *Yg = Y + ((int64_t)a * G + g) * plane;
        __syncthreads();
        for (int i = threadIdx.x; i < LH * LW; i += kBlock) {
            const int rr = i / LW;
            const int cc = i - rr * LW;
            const int v = v0 - C + rr;
            const int u = u0 - C + cc;
            tile[i] = (v >= 0 && v < nv && u >= 0 && u < nu) ? Yg[(int64_t)v * nu + u] : 0.0f;
        }
        __syncthreads();
        const float *kg = ker + g * K * K;
#pragma unroll
        for (int rr = 0; rr < ROWS + K - 1; ++rr) {
            float x[K];
#pragma unroll
            for (int j = 0; j < K; ++j) x[j] = tile[(wave * ROWS + rr) * LW + lane + j];
#pragma unroll
            for (int o = 0; o < ROWS; ++o) {
                const int i = rr - o;
                if (i >= 0 && i < K) {
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        acc[o] = fmaf(kg[(K - 1 - i) * K + (K - 1 - j)], x[j], acc[o]);
                }
            }
        }
    }
    const int u = u0 + lane;
#pragma unroll
    for (int o = 0; o < ROWS; ++o) {
        const int v = v0 + wave * ROWS + o;
        if (v < nv && u < nu) out[(int64_t)a * plane + (int64_t)v * nu + u] = acc[o];
    }
}

// Any odd k up to FCAT_MAX_PSF, runtime loops.
constexpr int kGenRows = 8;
constexpr int kGenLH = (kBlock / kWave) * kGenRows + FCAT_MAX_PSF - 1;
constexpr int kGenLW = kWave + FCAT_MAX_PSF - 1;

__global__ __launch_bounds__(kBlock) void k_psf_generic(const float *__restrict__ Y, int G, int nv, int nu,
                                                        const float *__restrict__ ker, int K,
                                                        float *__restrict__ out)
{
    constexpr int ROWS = kGenRows;
    constexpr int TU = kWave;
    constexpr int TV = (kBlock / kWave) * ROWS;
    __shared__ float tile[kGenLH * kGenLW];
    const int C = (K - 1) / 2;
    const int LW = TU + K - 1;
    const int LH = TV + K - 1;
    const int u0 = blockIdx.x * TU;
    const int v0 = blockIdx.y * TV;
    const int a = blockIdx.z;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t plane = (int64_t)nv * nu;
    float acc[ROWS];
#pragma unroll
    for (int o = 0; o < ROWS; ++o) acc[o] = 0.0f;
    for (int g = 0; g < G; ++g) {
        const float *Yg = Y + ((int64_t)a * G + g) * plane;
        __syncthreads();
        for (int i = threadIdx.x; i < LH * LW; i += kBlock) {
            const int rr = i / LW;
            const int cc = i - rr * LW;
            const int v = v0 - C + rr;
            const int u = u0 - C + cc;
            tile[i] = (v >= 0 && v < nv && u >= 0 && u < nu) ? Yg[(int64_t)v * nu + u] : 0.0f;
        }
        __syncthreads();
        const float *kg = ker + g * K * K;
#pragma unroll
        for (int o = 0; o < ROWS; ++o) {
            for (int i = 0; i < K; ++i) {
                const float *trow = tile + (wave * ROWS + o + i) * LW + lane;
                const float *krow = kg + (K - 1 - i) * K + (K - 1);
                for (int j = 0; j < K; ++j) acc[o] = fmaf(krow[-j], trow[j], acc[o]);
            }
        }
    }
    const int u = u0 + lane;
#pragma unroll
    for (int o = 0; o < ROWS; ++o) {
        const int v = v0 + wave * ROWS + o;
        if (v < nv && u < nu) out[(int64_t)a * plane + (int64_t)v * nu + u] = acc[o];
    }
}

// bricks[bz][by][bx] = the label shared by every voxel of the B x B x B brick
// (clipped at the grid edge), or -1 if they differ or the label is negative.
__global__ __launch_bounds__(kBlock) void k_build_bricks(const int8_t *__restrict__ labels, int nx, int ny,
                                                         int nz, int B, int nbx, int nby, int nbz,
                                                         int8_t *__restrict__ bricks)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= nbx * nby * nbz) return;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int x0 = bx * B, y0 = by * B, z0 = bz * B;
    const int x1 = min(x0 + B, nx), y1 = min(y0 + B, ny), z1 = min(z0 + B, nz);
    const int first = labels[((int64_t)z0 * ny + y0) * nx + x0];
    bool uniform = first >= 0;
    for (int z = z0; z < z1 && uniform; ++z)
        for (int y = y0; y < y1 && uniform; ++y) {
            const int8_t *row = labels + ((int64_t)z * ny + y) * nx;
            for (int x = x0; x < x1; ++x) uniform = uniform && row[x] == first;
        }
    bricks[b] = uniform ? (int8_t)first : (int8_t)-1;
}

int padded_blocks(int64_t waves)
{
    const int64_t nblk = (waves + (kBlock / kWave) - 1) / (kBlock / kWave);
    return (int)((nblk + kXcds - 1) / kXcds * kXcds);
}

}  // namespace

// ------------------------------------------------------------- launchers

hipError_t launch_prep_tables(const float *mu, const float *phi, const float *eta, const float *s_bin,
                              const SpecTables &t, float *muT, float *w, float *Wg, float *Wsg,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(k_prep_tables, dim3(1), dim3(kBlock), 0, stream, mu, phi, eta, s_bin, t, muT, w,
                       Wg, Wsg);
    return hipGetLastError();
}

hipError_t launch_project_rows(const TraceGeom &g, const int8_t *labels, const SpecTables &t,
                               const float *flood, const float *scatter, int a0, int n_ang, float *Y,
                               float *out, hipStream_t stream)
{
    const int wpr = (g.nu + kWave - 1) / kWave;
    const int64_t waves = (int64_t)n_ang * g.nv * wpr;
    const int nblk = padded_blocks(waves);
    switch (t.mp) {
    case 8:
        hipLaunchKernelGGL(k_project_rows<8>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, wpr, nblk, Y, out);
        break;
    case 16:
        hipLaunchKernelGGL(k_project_rows<16>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, wpr, nblk, Y, out);
        break;
    case 32:
        hipLaunchKernelGGL(k_project_rows<32>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, wpr, nblk, Y, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_build_bricks(const int8_t *labels, int nx, int ny, int nz, int B, int8_t *bricks,
                               hipStream_t stream)
{
    const int nbx = (nx + B - 1) / B, nby = (ny + B - 1) / B, nbz = (nz + B - 1) / B;
    const int nb = nbx * nby * nbz;
    hipLaunchKernelGGL(k_build_bricks, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, labels, nx,
                       ny, nz, B, nbx, nby, nbz, bricks);
    return hipGetLastError();
}

hipError_t launch_pathlengths(const TraceGeom &g, const int8_t *labels, int n_mat, int a0, int n_ang,
                              float *L, hipStream_t stream)
{
    const int wpr = (g.nu + kWave - 1) / kWave;
    const int64_t waves = (int64_t)n_ang * g.nv * wpr;
    const int nblk = padded_blocks(waves);
    if (n_mat <= 8)
        hipLaunchKernelGGL(k_pathlengths<8>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, wpr, nblk, L);
    else if (n_mat <= 16)
        hipLaunchKernelGGL(k_pathlengths<16>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, wpr, nblk, L);
    else
        hipLaunchKernelGGL(k_pathlengths<32>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, wpr, nblk, L);
    return hipGetLastError();
}

hipError_t launch_spectral(const float *L, int64_t n, const SpecTables &t, const float *i0,
                           const float *S, bool split, float *Y, hipStream_t stream)
{
    if (split) return hipErrorNotSupported;
    const unsigned nblk = (unsigned)((n + kBlock - 1) / kBlock);
    switch (t.mp) {
    case 8:
        hipLaunchKernelGGL(k_spectral<8>, dim3(nblk), dim3(kBlock), 0, stream, L, n, t, i0, S, Y);
        break;
    case 16:
        hipLaunchKernelGGL(k_spectral<16>, dim3(nblk), dim3(kBlock), 0, stream, L, n, t, i0, S, Y);
        break;
    case 32:
        hipLaunchKernelGGL(k_spectral<32>, dim3(nblk), dim3(kBlock), 0, stream, L, n, t, i0, S, Y);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_project_rows_split(const TraceGeom &, const int8_t *, const SpecTables &, const float *,
                                     const float *, int, int, float *, float *, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_psf(const float *Y, int n_ang, int G, int nv, int nu, const float *kernels, int k,
                      float *out, hipStream_t stream)
{
    constexpr int ROWS = 8;
    const dim3 grid((nu + kWave - 1) / kWave, (nv + 4 * ROWS - 1) / (4 * ROWS), n_ang);
    if (k == 15)
        hipLaunchKernelGGL((k_psf<15, ROWS>), grid, dim3(kBlock), 0, stream, Y, G, nv, nu, kernels, out);
    else
        hipLaunchKernelGGL(k_psf_generic, grid, dim3(kBlock), 0, stream, Y, G, nv, nu, kernels, k, out);
    return hipGetLastError();
}

hipError_t launch_check_labels(const int8_t *labels, int64_t n, int n_mat, int *flag, hipStream_t stream)
{
    const int64_t want = (n + kBlock - 1) / kBlock;
    const unsigned nblk = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    hipLaunchKernelGGL(k_check_labels, dim3(nblk), dim3(kBlock), 0, stream, labels, n, n_mat, flag);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float *x, int64_t n, int *flag, hipStream_t stream)
{
    const int64_t want = (n + kBlock - 1) / kBlock;
    const unsigned nblk = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    hipLaunchKernelGGL(k_check_finite, dim3(nblk), dim3(kBlock), 0, stream, x, n, flag);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_ints, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace fcat
