// gfx950 kernels of the polyenergetic cone-beam projector: the fused
// projector (traversal + spectral sum + scatter), path lengths only, the
// spectral sum on given path lengths, the optical spread, the brick map and
// input checks.  The shared device functions live in fcat_device.h.
#include "fcat_device.h"

#include <climits>

namespace fcat {
namespace {

// ------------------------------------------------------------ projector

template <int MP>
__global__ __launch_bounds__(kBlock) void k_project_rows(TraceGeom G, const int8_t *__restrict__ labels,
                                                         SpecTables T, const float *__restrict__ flood,
                                                         const float *__restrict__ scatter, int a0,
                                                         int n_ang, int nblk_pad, float *__restrict__ Y,
                                                         float *__restrict__ out)
{
    __shared__ float acc_all[(kBlock / kWave) * mat_acc_floats<MP>()];
    const int blk = xcd_block(nblk_pad);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blk * (kBlock / kWave) + wave;
    if (gw >= n_ang * tiles_per_angle(G)) return;
    const PixelOf px = pixel_of(G, gw, lane);
    const int al = px.al, iv = px.iv, iu = px.iu;
    const int a = a0 + al;
    const bool valid = px.valid;

    double st, ct;
    angle_trig(G, a, st, ct);
    float L[MP];
    Ray r{};
    const bool hit = valid && setup_ray(G, ct, st, iv, iu, r);
    trace_bricks<MP>(r, hit, G, G.labels_bm, G.bricks, acc_all + wave * mat_acc_floats<MP>(), L);
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
    flag_nonfinite(G.bad, i0, sc);
}

template <int MP>
__global__ __launch_bounds__(kBlock) void k_pathlengths(TraceGeom G, const int8_t *__restrict__ labels,
                                                        int n_mat, int a0, int n_ang, int nblk_pad,
                                                        float *__restrict__ Lout)
{
    __shared__ float acc_all[(kBlock / kWave) * mat_acc_floats<MP>()];
    const int blk = xcd_block(nblk_pad);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blk * (kBlock / kWave) + wave;
    if (gw >= n_ang * tiles_per_angle(G)) return;
    const PixelOf px = pixel_of(G, gw, lane);
    const int al = px.al, iv = px.iv, iu = px.iu;
    const bool valid = px.valid;
    double st, ct;
    angle_trig(G, a0 + al, st, ct);
    float L[MP];
    Ray r{};
    const bool hit = valid && setup_ray(G, ct, st, iv, iu, r);
    trace_bricks<MP>(r, hit, G, G.labels_bm, G.bricks, acc_all + wave * mat_acc_floats<MP>(), L);
    if (!valid) return;
    float *dst = Lout + (((int64_t)al * G.nv + iv) * G.nu + iu) * n_mat;
#pragma unroll
    for (int m = 0; m < MP; ++m)
        if (m < n_mat) dst[m] = L[m];
}

// Voxel segments of Siddon's method on the ray to pixel (iv, iu): one per
// voxel between entry and exit, 1 + sum over axes of |i_exit - i_entry|, the
// two voxels taken by floor of the FP64 entry and exit points (clamped to
// the grid); 0 for a ray that misses.  The unit of work the walk is priced
// against, counted here so that no host pass over every ray is needed.
__device__ uint32_t siddon_segments(const TraceGeom &G, double ct, double st, int iv, int iu)
{
    const double pu = ((double)iu - G.cu) * G.du + G.off_u;
    const double pv = ((double)iv - G.cv) * G.dv + G.off_v;
    const double s[3] = {G.sid * ct, G.sid * st, 0.0};
    const double p[3] = {-G.back * ct - pu * st, -G.back * st + pu * ct, pv};
    double d[3], amin = 0.0, amax = 1.0;
    bool inside = true;
    for (int ax = 0; ax < 3; ++ax) {
        d[ax] = p[ax] - s[ax];
        const double lo = G.lo[ax], hi = G.lo[ax] + G.n[ax] * G.h[ax];
        if (d[ax] == 0.0) {
            inside = inside && s[ax] >= lo && s[ax] < hi;
        } else {
            const double a0 = (lo - s[ax]) / d[ax], a1 = (hi - s[ax]) / d[ax];
            amin = fmax(amin, fmin(a0, a1));
            amax = fmin(amax, fmax(a0, a1));
        }
    }
    if (!inside || !(amax > amin)) return 0;
    uint32_t n = 1;
    for (int ax = 0; ax < 3; ++ax) {
        const int i0 = min(max((int)floor((s[ax] + amin * d[ax] - G.lo[ax]) * G.inv_h[ax]), 0), G.n[ax] - 1);
        const int i1 = min(max((int)floor((s[ax] + amax * d[ax] - G.lo[ax]) * G.inv_h[ax]), 0), G.n[ax] - 1);
        n += (uint32_t)abs(i1 - i0);
    }
    return n;
}

// Step counts of the walk over angles [a0, a0 + n_ang): counts[0] rays that
// meet the grid, [1] brick steps, [2] mixed bricks entered, [3] voxel steps,
// [4] wavefront iterations of the voxel loop times 64 (lane slots), [5]
// Siddon voxel segments.  Per-lane counts are summed over the wavefront with
// shuffles and over the workgroup in LDS, then one 64-bit atomic per
// workgroup and counter (every add goes to one of six words, so their
// number sets much of the call's time).
template <int MP>
__global__ __launch_bounds__(kBlock) void k_walk_stats(TraceGeom G, int a0, int n_ang, int nblk_pad,
                                                       unsigned long long *__restrict__ counts)
{
    __shared__ float acc_all[(kBlock / kWave) * mat_acc_floats<MP>()];
    __shared__ unsigned long long part[kBlock / kWave][kWalkCounts];
    const int blk = xcd_block(nblk_pad);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blk * (kBlock / kWave) + wave;
    unsigned long long v[kWalkCounts] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    // wave-uniform: a wavefront past the last tile adds zeros but still
    // reaches the workgroup barrier below
    if (gw < n_ang * tiles_per_angle(G)) {
        const PixelOf px = pixel_of(G, gw, lane);
        double st, ct;
        angle_trig(G, a0 + px.al, st, ct);
        float L[MP];
        Ray r{};
        const bool hit = px.valid && setup_ray(G, ct, st, px.iv, px.iu, r);
        StepCount c;
        trace_bricks<MP>(r, hit, G, G.labels_bm, G.bricks, acc_all + wave * mat_acc_floats<MP>(), L, c);
        const uint32_t segs = px.valid ? siddon_segments(G, ct, st, px.iv, px.iu) : 0u;
        v[0] = hit ? 1ull : 0ull;
        v[1] = hit ? (unsigned long long)c.bricks : 0ull;
        v[2] = c.mixed_bricks;
        v[3] = c.voxels;
        v[4] = 64ull * c.wave_voxel_iters;
        v[5] = segs;
#pragma unroll
        for (int k = 0; k < kWalkCounts; ++k)
            for (int off = kWave / 2; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kWalkCounts; ++k) part[wave][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < kWalkCounts) {
        unsigned long long sum = 0ull;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) sum += part[w][threadIdx.x];
        if (sum) atomicAdd(counts + threadIdx.x, sum);
    }
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
                                                        float *__restrict__ Wg, float *__restrict__ Wsg,
                                                        const float *__restrict__ psf_k, int n_psf, int *bad)
{
    // The tables are read here once per call, so this is where their
    // finiteness is checked (bad[1] |= 1), together with the spread kernels.
    bool nonfinite = false;
    for (int e = threadIdx.x; e < T.E; e += kBlock) {
        const float p = phi[e], q = eta[e];
        w[e] = p * q;
        nonfinite = nonfinite || !isfinite(p) || !isfinite(q) || (s_bin && !isfinite(s_bin[e]));
        for (int m = 0; m < T.mp; ++m) {
            const float v = m < T.M ? mu[(int64_t)m * T.E + e] : 0.0f;
            nonfinite = nonfinite || !isfinite(v);
            muT[e * T.mp + m] = v;
            // the same table in base 2 follows it: exp(-mu L) = 2^-(mu log2(e) L)
            muT[(T.E + e) * T.mp + m] = (float)((double)v * 1.44269504088896340736);
        }
    }
    if (bad) {
        for (int i = threadIdx.x; i < n_psf; i += kBlock) nonfinite = nonfinite || !isfinite(psf_k[i]);
        if (__syncthreads_or(nonfinite) && threadIdx.x == 0) atomicOr(bad + 1, 1);
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

// The same convolution with a 4 x 4 output block per lane: lane l of
// wavefront w owns columns 4l .. 4l + 3 and rows 4w .. 4w + 3 of a 256 x (4 * kP4Waves)
// output tile.  The LDS tile starts 8 columns left of the outputs, so each
// 16-byte global load of an aligned column group is one aligned 16-byte LDS
// store (storing the four values one by one, 4 columns apart across the
// lanes, met each LDS bank four times: 2% slower on the head workload).
// For each input row a lane reads the tile columns 4l .. 4l + NX - 1 with
// aligned 16-byte LDS loads (immediate offsets, no address arithmetic) and
// feeds its K + 3 inputs, from column 4l + 8 - C on, to up to 4 x 4 outputs.  The flipped kernel of the group is staged in
// LDS beside the tile and each kernel row is read into vector registers
// (a broadcast LDS read) where it is used: an FMA whose operands are all
// vector registers can issue at up to about 1.6 times the rate of one that
// reads a scalar register, given enough wavefronts per SIMD.
constexpr int kP4Cols = 4 * kWave;              // 256 output columns per tile
constexpr int kP4Waves = 8;                     // wavefronts per workgroup (4 and 16 measured slower)
constexpr int kP4Rows = 4 * kP4Waves;           // output rows per tile
constexpr int kPsfStore = 0, kPsfRatio = 1, kPsfUpdate = 2;

// EPI selects what is stored for a convolution value c (Richardson-Lucy
// steps fused into the convolution):
//   kPsfStore:  out = c
//   kPsfRatio:  out = c > 0 ? aux[i] / c : 0        (aux = the data d)
//   kPsfUpdate: out = out[i] * c / norm[pixel]     (out = the iterate u, in place)
template <int K, int NW, int EPI>
__global__ __launch_bounds__(NW * kWave) void k_psf4(const float *__restrict__ Y, int G, int nv, int nu,
                                                     const float *__restrict__ ker, float *out,
                                                     const float *aux, const float *__restrict__ norm)
{
    constexpr int C = (K - 1) / 2;
    constexpr int X0 = 8 - C;                     // first tile column a lane uses, past 4 l
    constexpr int NX = (X0 + K + 3 + 3) / 4 * 4;  // inputs read per row, a multiple of 4
    constexpr int LW = kP4Cols + NX - 4;          // tile width (covers the last lane's reads)
    constexpr int ROWS = 4 * NW;
    constexpr int LH = ROWS + K - 1;
    constexpr int NT = NW * kWave;
    constexpr int KW = (K + 3) / 4 * 4;           // kernel row stride in LDS (zero-padded)
    static_assert(LW % 4 == 0, "aligned rows");
    static_assert(K * KW <= NT, "one thread per staged weight");
    static_assert(C <= 8, "the aligned tile loads start at most 8 columns left of the tile");
    __shared__ __align__(16) float tile[LH * LW];
    __shared__ __align__(16) float wl[K * KW];   // wl[i][j] = K_g[K-1-i][K-1-j]
    const int u0 = blockIdx.x * kP4Cols;
    const int v0 = blockIdx.y * ROWS;
    const int a = blockIdx.z;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t plane = (int64_t)nv * nu;
    const bool vec_loads = (nu & 3) == 0 && (reinterpret_cast<uintptr_t>(Y) & 15) == 0;
    float acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0f;

    for (int g = 0; g < G; ++g) {
        const float *Yg = Y + ((int64_t)a * G + g) * plane;
        __syncthreads();
        if (vec_loads) {
            // 16-byte global loads from the aligned columns u0 - 8 + 4m, each
            // value written to tile column u - (u0 - C); with nu a multiple of 4
            // a group is inside the detector or not at all
            constexpr int G4 = LW / 4;
            for (int i = threadIdx.x; i < LH * G4; i += NT) {
                const int rr = i / G4;
                const int m = i - rr * G4;
                const int v = v0 - C + rr;
                const int u = u0 - 8 + 4 * m;
                float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
                if (v >= 0 && v < nv && u >= 0 && u < nu)
                    y = *reinterpret_cast<const float4 *>(Yg + (int64_t)v * nu + u);
                *reinterpret_cast<float4 *>(tile + rr * LW + 4 * m) = y;
            }
        } else {
            for (int i = threadIdx.x; i < LH * LW; i += NT) {
                const int rr = i / LW;
                const int cc = i - rr * LW;
                const int v = v0 - C + rr;
                const int u = u0 - 8 + cc;
                tile[i] = (v >= 0 && v < nv && u >= 0 && u < nu) ? Yg[(int64_t)v * nu + u] : 0.0f;
            }
        }
        if (threadIdx.x < K * KW) {
            const int i = threadIdx.x / KW, j = threadIdx.x - i * KW;
            wl[threadIdx.x] = j < K ? ker[(int64_t)g * K * K + (K - 1 - i) * K + (K - 1 - j)] : 0.0f;
        }
        __syncthreads();
        const float *trow = tile + (4 * wave) * LW + 4 * lane;
#pragma unroll
        for (int rr = 0; rr < K + 3; ++rr) {
            float x[NX];
#pragma unroll
            for (int j = 0; j < NX; j += 4) {
                const float4 v4 = *reinterpret_cast<const float4 *>(trow + rr * LW + j);
                x[j] = v4.x;
                x[j + 1] = v4.y;
                x[j + 2] = v4.z;
                x[j + 3] = v4.w;
            }
            // the end values are not products' operands; using them here
            // keeps each row read as whole aligned 16-byte LDS loads
            __asm__ volatile("" ::"v"(x[0]), "v"(x[NX - 1]));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = rr - r;
                if (i >= 0 && i < K) {
                    // the kernel row is read again for every output row: the
                    // compiler barrier stops it from keeping four rows live,
                    // which would cost about 36 registers and with them occupancy
                    __asm__ volatile("" ::: "memory");
                    float w[KW];
#pragma unroll
                    for (int j = 0; j < KW; j += 4) {
                        const float4 w4 = *reinterpret_cast<const float4 *>(wl + i * KW + j);
                        w[j] = w4.x;
                        w[j + 1] = w4.y;
                        w[j + 2] = w4.z;
                        w[j + 3] = w4.w;
                    }
#pragma unroll
                    for (int j = 0; j < K; ++j)
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(w[j], x[X0 + c + j], acc[r][c]);
                }
            }
        }
    }
    const int ub = u0 + 4 * lane;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int v = v0 + 4 * wave + r;
        if (v >= nv) continue;
        const int64_t pix = (int64_t)v * nu + ub;
        const int64_t at = (int64_t)a * plane + pix;
        float *o = out + at;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (ub + c >= nu) break;
            if (EPI == kPsfRatio) {
                const float d = aux[at + c];
                acc[r][c] = acc[r][c] > 0.0f ? d / acc[r][c] : 0.0f;
            } else if (EPI == kPsfUpdate) {
                acc[r][c] = o[c] * acc[r][c] / norm[pix + c];
            }
        }
        if ((nu & 3) == 0 && ub + 3 < nu) {
            *reinterpret_cast<float4 *>(o) = make_float4(acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (ub + c < nu) o[c] = acc[r][c];
        }
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

// Brick map and brick-major copy of the labels.  One workgroup per brick:
// the threads copy the brick's labels (positions past the grid edge get the
// nearest voxel inside it) into labels_bm[brick][z][y][x], and the brick is
// uniform when every voxel inside the grid carries the same non-negative
// label.  bricks[b] holds that label, or -1.  Every label is read here once
// per call, so with bad non-null a label outside 0..n_mat-1 sets bad[0].
constexpr int kBuildThreads = kBrickVox < 512 ? kBrickVox : 512;

__global__ __launch_bounds__(kBuildThreads) void k_build_bricks(const int8_t *__restrict__ labels, int nx, int ny,
                                                                int nz, int nbx, int nby,
                                                                int8_t *__restrict__ bricks,
                                                                int8_t *__restrict__ labels_bm, int n_mat, int *bad)
{
    const int b = blockIdx.x;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    __shared__ int first;
    if (threadIdx.x == 0)
        first = labels[((int64_t)(bz * kBrickEdge) * ny + by * kBrickEdge) * nx + bx * kBrickEdge];
    __syncthreads();
    const int f = first;
    bool diff = f < 0;
    bool out_of_range = false;
    for (int i = threadIdx.x; i < kBrickVox; i += kBuildThreads) {
        const int lx = i & (kBrickEdge - 1);
        const int ly = (i / kBrickEdge) & (kBrickEdge - 1);
        const int lz = i / (kBrickEdge * kBrickEdge);
        const int x = bx * kBrickEdge + lx, y = by * kBrickEdge + ly, z = bz * kBrickEdge + lz;
        const bool in = x < nx && y < ny && z < nz;
        const int v = labels[((int64_t)min(z, nz - 1) * ny + min(y, ny - 1)) * nx + min(x, nx - 1)];
        labels_bm[(int64_t)b * kBrickVox + i] = (int8_t)v;
        diff = diff || (in && v != f);
        out_of_range = out_of_range || (in && (v < 0 || v >= n_mat));
    }
    const bool mixed = __syncthreads_or(diff);
    if (bad && __syncthreads_or(out_of_range) && threadIdx.x == 0) atomicOr(bad, 1);
    if (threadIdx.x == 0) bricks[b] = mixed ? (int8_t)-1 : (int8_t)f;
    // the first and the last workgroup fill the padding before and after the copy
    if (b == 0)
        for (uint32_t i = threadIdx.x; i < kLabelPad; i += kBuildThreads) labels_bm[(int64_t)i - kLabelPad] = (int8_t)-1;
    if (b == (int)gridDim.x - 1)
        for (uint32_t i = threadIdx.x; i < kLabelPad; i += kBuildThreads)
            labels_bm[(int64_t)gridDim.x * kBrickVox + i] = (int8_t)-1;
}

// The background box (TraceGeom::clip) from the brick map: the label of
// brick 0 when that brick is uniform, and the brick-aligned box of every
// brick that is not uniform with it.  One workgroup.
__global__ __launch_bounds__(kBlock) void k_clip_box(const int8_t *__restrict__ bricks, int nbx, int nby, int nbz,
                                                     int nx, int ny, int nz, int *__restrict__ clip)
{
    __shared__ int box[6];
    if (threadIdx.x < 3) box[threadIdx.x] = INT_MAX;
    else if (threadIdx.x < 6) box[threadIdx.x] = -1;
    __syncthreads();
    const int bg = bricks[0];   // -1 if brick 0 is mixed: then every brick is in the box
    const int nb = nbx * nby * nbz;
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-1, -1, -1};
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        if (bg >= 0 && bricks[b] == bg) continue;
        const int c[3] = {b % nbx, (b / nbx) % nby, b / (nbx * nby)};
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], c[a]);
            hi[a] = max(hi[a], c[a]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        atomicMin(&box[a], lo[a]);
        atomicMax(&box[3 + a], hi[a]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int n[3] = {nx, ny, nz};
        const bool any = box[3] >= 0;
        clip[0] = bg;
        for (int a = 0; a < 3; ++a) {
            clip[1 + a] = any ? box[a] * kBrickEdge : 0;
            clip[4 + a] = any ? min((box[3 + a] + 1) * kBrickEdge, n[a]) : 0;
        }
        clip[7] = any ? 1 : 0;
    }
}

// Cosine and sine of every angle, once per projector call (the walk kernels
// read them per wavefront instead of evaluating them per lane).
__global__ __launch_bounds__(kBlock) void k_trig_table(TraceGeom G, double *__restrict__ trig)
{
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= G.n_angles) return;
    double st, ct;
    sincos(angle_of(G, a), &st, &ct);
    trig[2 * a] = ct;
    trig[2 * a + 1] = st;
}

}  // namespace

// ------------------------------------------------------------- launchers

hipError_t launch_trig_table(const TraceGeom &g, double *trig, hipStream_t stream)
{
    hipLaunchKernelGGL(k_trig_table, dim3((g.n_angles + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, g, trig);
    return hipGetLastError();
}

hipError_t launch_prep_tables(const float *mu, const float *phi, const float *eta, const float *s_bin,
                              const SpecTables &t, float *muT, float *w, float *Wg, float *Wsg,
                              hipStream_t stream, const InputCheck &chk)
{
    hipLaunchKernelGGL(k_prep_tables, dim3(1), dim3(kBlock), 0, stream, mu, phi, eta, s_bin, t, muT, w,
                       Wg, Wsg, chk.psf, chk.n_psf, chk.bad);
    return hipGetLastError();
}

hipError_t launch_project_rows(const TraceGeom &g, const int8_t *labels, const SpecTables &t,
                               const float *flood, const float *scatter, int a0, int n_ang, float *Y,
                               float *out, hipStream_t stream)
{
    const int64_t waves = (int64_t)n_ang * tiles_per_angle_host(g);
    const int nblk = padded_blocks(waves);
    switch (t.mp) {
    case 8:
        hipLaunchKernelGGL(k_project_rows<8>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, nblk, Y, out);
        break;
    case 10:
        hipLaunchKernelGGL(k_project_rows<10>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, nblk, Y, out);
        break;
    case 12:
        hipLaunchKernelGGL(k_project_rows<12>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, nblk, Y, out);
        break;
    case 16:
        hipLaunchKernelGGL(k_project_rows<16>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, nblk, Y, out);
        break;
    case 32:
        hipLaunchKernelGGL(k_project_rows<32>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, t, flood,
                           scatter, a0, n_ang, nblk, Y, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_build_bricks(const int8_t *labels, int nx, int ny, int nz, int8_t *bricks, int8_t *labels_bm,
                               int *clip, hipStream_t stream, int n_mat, int *bad)
{
    const int nbx = (nx + kBrickEdge - 1) / kBrickEdge, nby = (ny + kBrickEdge - 1) / kBrickEdge;
    const int nbz = (nz + kBrickEdge - 1) / kBrickEdge;
    hipLaunchKernelGGL(k_build_bricks, dim3(nbx * nby * nbz), dim3(kBuildThreads), 0, stream, labels, nx, ny, nz, nbx,
                       nby, bricks, labels_bm, n_mat, bad);
    hipLaunchKernelGGL(k_clip_box, dim3(1), dim3(kBlock), 0, stream, bricks, nbx, nby, nbz, nx, ny, nz, clip);
    return hipGetLastError();
}

hipError_t launch_pathlengths(const TraceGeom &g, const int8_t *labels, int n_mat, int a0, int n_ang,
                              float *L, hipStream_t stream)
{
    const int64_t waves = (int64_t)n_ang * tiles_per_angle_host(g);
    const int nblk = padded_blocks(waves);
    if (n_mat <= 8)
        hipLaunchKernelGGL(k_pathlengths<8>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, nblk, L);
    else if (n_mat <= 10)
        hipLaunchKernelGGL(k_pathlengths<10>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, nblk, L);
    else if (n_mat <= 12)
        hipLaunchKernelGGL(k_pathlengths<12>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, nblk, L);
    else if (n_mat <= 16)
        hipLaunchKernelGGL(k_pathlengths<16>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, nblk, L);
    else
        hipLaunchKernelGGL(k_pathlengths<32>, dim3(nblk), dim3(kBlock), 0, stream, g, labels, n_mat, a0,
                           n_ang, nblk, L);
    return hipGetLastError();
}

hipError_t launch_walk_stats(const TraceGeom &g, int a0, int n_ang, unsigned long long *counts, hipStream_t stream)
{
    const int64_t waves = (int64_t)n_ang * tiles_per_angle_host(g);
    const int nblk = padded_blocks(waves);
    hipLaunchKernelGGL(k_walk_stats<8>, dim3(nblk), dim3(kBlock), 0, stream, g, a0, n_ang, nblk, counts);
    return hipGetLastError();
}

hipError_t launch_spectral(const float *L, int64_t n, const SpecTables &t, const float *i0,
                           const float *S, float *Y, hipStream_t stream)
{
    const unsigned nblk = (unsigned)((n + kBlock - 1) / kBlock);
    switch (t.mp) {
    case 8:
        hipLaunchKernelGGL(k_spectral<8>, dim3(nblk), dim3(kBlock), 0, stream, L, n, t, i0, S, Y);
        break;
    case 10:
        hipLaunchKernelGGL(k_spectral<10>, dim3(nblk), dim3(kBlock), 0, stream, L, n, t, i0, S, Y);
        break;
    case 12:
        hipLaunchKernelGGL(k_spectral<12>, dim3(nblk), dim3(kBlock), 0, stream, L, n, t, i0, S, Y);
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


hipError_t launch_psf(const float *Y, int n_ang, int G, int nv, int nu, const float *kernels, int k,
                      float *out, hipStream_t stream)
{
    // 4 rows per lane: with 8 the 8 x 15 kernel weights live at once exceed
    // the scalar registers and spill through VGPR lanes (measured 41 vs 50
    // TFLOP/s on the contrast workload)
    constexpr int ROWS = 4;
    constexpr int TV = (kBlock / kWave) * ROWS;
    constexpr int TVG = (kBlock / kWave) * kGenRows;
    if (k == 15) {
        const dim3 grid((nu + kP4Cols - 1) / kP4Cols, (nv + kP4Rows - 1) / kP4Rows, n_ang);
        hipLaunchKernelGGL((k_psf4<15, kP4Waves, kPsfStore>), grid, dim3(kP4Waves * kWave), 0, stream, Y, G, nv, nu,
                           kernels, out, nullptr, nullptr);
    } else if (k == 5) {
        const dim3 grid((nu + kWave - 1) / kWave, (nv + TV - 1) / TV, n_ang);
        hipLaunchKernelGGL((k_psf<5, ROWS>), grid, dim3(kBlock), 0, stream, Y, G, nv, nu, kernels, out);
    } else {
        const dim3 grid((nu + kWave - 1) / kWave, (nv + TVG - 1) / TVG, n_ang);
        hipLaunchKernelGGL(k_psf_generic, grid, dim3(kBlock), 0, stream, Y, G, nv, nu, kernels, k, out);
    }
    return hipGetLastError();
}

hipError_t launch_psf_rl(int step, const float *Y, int n_ang, int nv, int nu, const float *kernel, int k,
                         float *out, const float *data, const float *norm, hipStream_t stream)
{
    if (k != 15 || (step != 1 && step != 2)) return hipErrorInvalidValue;
    const dim3 grid((nu + kP4Cols - 1) / kP4Cols, (nv + kP4Rows - 1) / kP4Rows, n_ang);
    if (step == 1)
        hipLaunchKernelGGL((k_psf4<15, kP4Waves, kPsfRatio>), grid, dim3(kP4Waves * kWave), 0, stream, Y, 1, nv, nu,
                           kernel, out, data, nullptr);
    else
        hipLaunchKernelGGL((k_psf4<15, kP4Waves, kPsfUpdate>), grid, dim3(kP4Waves * kWave), 0, stream, Y, 1, nv, nu,
                           kernel, out, nullptr, norm);
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
