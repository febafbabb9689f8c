// Split-precision form of the L . mu contraction on the gfx950 matrix cores.
//
// The optical depth P_e = sum_m mu[m][e] L_m (one projection per energy,
// Sec. II.F) is evaluated as
//     mu_hi L_hi + mu_lo L_hi + mu_hi L_lo
// with x_hi = bf16(x) (round to nearest even) and x_lo = bf16(x - x_hi).
// BF16 x BF16 products are exact in FP32 and v_mfma_f32_16x16x32_bf16
// accumulates in FP32; the dropped lo x lo term and the rounding of the two
// residuals leave a relative error of order 3 * 2^-16 per product, so
// |dP| <~ 4.6e-5 P and |dY / Y| <~ 4.6e-5 P_eff.
//
// One wavefront contracts the 64 rays of its lanes: each lane writes the
// BF16 k-vector [L_hi | L_hi | L_lo] of its ray to LDS; the B operands (32 k
// x 16 rays) are read back in matrix-core lane order; the A operands
// (16 energies x 32 k, prepared once per call) come from the workspace.
// With energies on the rows, a lane receives 4 energies of one ray per
// tile, applies w_e exp(-P_e) and sums them; tiles never straddle two
// energy groups (each group is padded to whole tiles with zero weight), so
// a group sum is the lane's partial sums reduced over the four lane
// quarters that hold the same ray.
//
// The optical spread (Sec. II.G, Eq. 1) of the split form runs on the
// matrix cores as well; see k_psf_split below.
#include "fcat_device.h"

namespace fcat {
namespace {

// One BF16 row of K = 32 NKB values per ray, unpadded; the 16-byte chunk c of
// row r is stored at chunk c ^ swz(r).  A matrix-core operand read takes 16
// consecutive rows (lane & 15) and two chunks per row in each half wavefront;
// with 128 four-byte LDS banks, 16-byte reads by 32 lanes are free of
// conflicts when those 32 chunks are distinct modulo 512 bytes.  Rows of 64
// and 96 bytes repeat every 8 rows and rows of 128 bytes every 4 rows, so
// the swizzle moves the later rows onto other chunks.  (The earlier padded
// stride of K + 8 left 13-17% of the walk kernel's LDS cycles in conflicts;
// removing them did not change its time, which the walk decides.)
template <int NKB>
constexpr int split_row_stride() { return NKB * 32; }   // BF16 units

template <int NKB>
__device__ __forceinline__ int split_swz(int r)
{
    return NKB == 2 ? ((r >> 2) & 3) << 1 : ((r >> 3) & 1) << 1;
}

// Offset (BF16 units) of value k of row r.
template <int NKB>
__device__ __forceinline__ int split_at(int r, int k)
{
    return r * split_row_stride<NKB>() + ((((k >> 3) ^ split_swz<NKB>(r))) << 3) + (k & 7);
}

// Group sums sum_{e in g} w_e exp(-P_e) of the 64 rays of the calling
// wavefront (one per lane, path lengths L); emit(g, value) receives the
// lane's own ray.  Every lane of the wavefront must be active.
template <int MP, int NKB, typename Emit>
__device__ __forceinline__ void split_group_sums(const float (&L)[MP], int M, int G, const SplitTables &S,
                                                 uint16_t *lds, Emit emit)
{
    constexpr int KW = NKB * 32;
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int k = 0; k < KW; k += 8) *reinterpret_cast<uint4 *>(lds + split_at<NKB>(lane, k)) = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int m = 0; m < MP; ++m) {
        if (m < M) {
            const uint32_t hi = bf16_rne(L[m]);
            const uint32_t lo = bf16_rne(L[m] - bf16_value(hi));
            lds[split_at<NKB>(lane, m)] = (uint16_t)hi;
            lds[split_at<NKB>(lane, M + m)] = (uint16_t)hi;
            lds[split_at<NKB>(lane, 2 * M + m)] = (uint16_t)lo;
        }
    }
    // the rows are read by other lanes of this wavefront
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const int q = lane >> 4;
    bf16x8 bfrag[4][NKB];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
            bfrag[c][kb] = *reinterpret_cast<const bf16x8 *>(lds + split_at<NKB>(16 * c + (lane & 15), kb * 32 + 8 * q));

    for (int g = 0; g < G; ++g) {
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int t = S.gtile[g]; t < S.gtile[g + 1]; ++t) {
            const float4 w4 = *reinterpret_cast<const float4 *>(S.wtile + t * 16 + 4 * q);
            bf16x8 a[NKB];
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                const uint4 raw = S.afrag[(t * NKB + kb) * kWave + lane];
                a[kb] = __builtin_bit_cast(bf16x8, raw);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kb = 0; kb < NKB; ++kb)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kb], bfrag[c][kb], acc, 0, 0, 0);
                part[c] += w4.x * __expf(-acc[0]) + w4.y * __expf(-acc[1]) + w4.z * __expf(-acc[2]) +
                           w4.w * __expf(-acc[3]);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            part[c] += __shfl_xor(part[c], 16);
            part[c] += __shfl_xor(part[c], 32);
        }
        const float mine = q == 0 ? part[0] : (q == 1 ? part[1] : (q == 2 ? part[2] : part[3]));
        emit(g, mine);
    }
}

template <int MP, int NKB>
__global__ __launch_bounds__(kBlock) void k_project_rows_split(TraceGeom G, SpecTables T, SplitTables S,
                                                               const float *__restrict__ flood,
                                                               const float *__restrict__ scatter, int a0,
                                                               int n_ang, int nblk_pad,
                                                               float *__restrict__ Y, float *__restrict__ out)
{
    // per wavefront: the traversal's material accumulators, then (after the
    // walk, same wavefront only) the rows of the split contraction
    constexpr int kRowBytes = kWave * split_row_stride<NKB>() * 2;
    constexpr int kAccBytes = mat_acc_floats<MP>() * 4;
    constexpr int kWaveBytes = kRowBytes > kAccBytes ? kRowBytes : kAccBytes;
    static_assert(kWaveBytes % 16 == 0, "16-byte aligned rows in every wavefront's block");
    __shared__ __align__(16) uint8_t lds_raw[(kBlock / kWave) * kWaveBytes];
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
    uint8_t *lds_wave = lds_raw + wave * kWaveBytes;
    trace_bricks<MP>(r, hit, G, G.labels_bm, G.bricks, reinterpret_cast<float *>(lds_wave), L);
    const bool any_hit = __ballot(hit) != 0;
    wave_sync_lds();

    const int64_t plane = (int64_t)G.nu * G.nv;
    const int64_t pix = (int64_t)min(iv, G.nv - 1) * G.nu + min(iu, G.nu - 1);   // all lanes take part
    const float i0 = flood ? flood[pix] : 1.0f;
    const float sc = scatter ? scatter[(int64_t)a * plane + pix] : 0.0f;
    float total = 0.0f;
    auto emit = [&](int g, float prim) {
        const float y = fmaf(i0, prim, T.Wsg[g] * sc);
        if (Y) {
            if (valid) Y[((int64_t)al * T.G + g) * plane + pix] = y;
        } else {
            total += y;
        }
    };
    if (any_hit) {
        split_group_sums<MP, NKB>(L, T.M, T.G, S, reinterpret_cast<uint16_t *>(lds_wave), emit);
    } else {
        for (int g = 0; g < T.G; ++g) emit(g, T.Wg[g]);
    }
    if (!Y && valid) out[(int64_t)a * plane + pix] = total;
    flag_nonfinite(G.bad, i0, sc);
}

template <int MP, int NKB>
__global__ __launch_bounds__(kBlock) void k_spectral_split(const float *__restrict__ Lin, int64_t n, SpecTables T,
                                                           SplitTables S, const float *__restrict__ i0,
                                                           const float *__restrict__ Sc, float *__restrict__ Y)
{
    __shared__ __align__(16) uint16_t lds_all[(kBlock / kWave) * kWave * split_row_stride<NKB>()];
    const int wave = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < n;
    float L[MP];
#pragma unroll
    for (int m = 0; m < MP; ++m) L[m] = (valid && m < T.M) ? Lin[r * T.M + m] : 0.0f;
    const float f = (valid && i0) ? i0[r] : 1.0f;
    const float sc = (valid && Sc) ? Sc[r] : 0.0f;
    auto emit = [&](int g, float prim) {
        if (valid) Y[(int64_t)g * n + r] = fmaf(f, prim, T.Wsg[g] * sc);
    };
    split_group_sums<MP, NKB>(L, T.M, T.G, S, lds_all + wave * kWave * split_row_stride<NKB>(), emit);
}

// A operands and weights of the split contraction (see SplitTables).
__global__ __launch_bounds__(kBlock) void k_prep_split(const float *__restrict__ mu, SpecTables T, SplitTables S,
                                                       uint4 *__restrict__ afrag, float *__restrict__ wtile)
{
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= S.T * S.nkb * kWave) return;
    const int lane = idx % kWave;
    const int kb = (idx / kWave) % S.nkb;
    const int t = idx / (kWave * S.nkb);
    int g = 0;
    while (g + 1 < T.G && S.gtile[g + 1] <= t) ++g;
    const int row = lane & 15;
    const int e = T.gstart[g] + 16 * (t - S.gtile[g]) + row;
    const bool ev = e < T.gstart[g + 1];
    uint32_t h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = kb * 32 + 8 * (lane >> 4) + j;
        uint32_t v = 0u;
        if (ev && k < 3 * T.M) {
            const int m = k % T.M;
            const float x = mu[(int64_t)m * T.E + e];
            const uint32_t hi = bf16_rne(x);
            v = (k >= T.M && k < 2 * T.M) ? bf16_rne(x - bf16_value(hi)) : hi;
        }
        h[j] = v;
    }
    afrag[idx] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    if (kb == 0 && lane < 16) wtile[t * 16 + lane] = ev ? T.w[e] : 0.0f;
}

// ---------------------------------------------------------- split PSF
//
// out[v][u] = sum_g sum_{p,q} K_g[p][q] Y_g[v - p + c][u - q + c] (true
// convolution, zero outside the detector, c = (k - 1) / 2).  For one kernel
// row p, sixteen consecutive outputs of a detector row depend on 16 + k - 1
// consecutive inputs, so the row convolution is a 16 x 32 by 32 x 16 matrix
// product: A[r][j] = Y_g[v0 + r - p + c][u0 - 8 + j] (16 output rows r; the
// tile starts 8 columns left of the outputs, so that its global loads are
// 16-byte aligned), B_{g,p}[j][t] = K_g[p][t + c + 8 - j] where
// 0 <= t + c + 8 - j < k, else 0 (a banded Toeplitz block, built once per
// call; for odd k <= 17 the band lies inside the 32 columns).  Both operands are split into
// BF16 hi/lo parts and each product is formed as A_hi B_hi + A_lo B_hi +
// A_hi B_lo with FP32 accumulation over p, g and the three terms.  Every
// term is non-negative, so the relative error of an output is that of a
// single product, below 3 * 2^-17.  A workgroup computes a 64 x 64 output
// tile: wavefront w the rows 16w .. 16w + 15, as four 16 x 16 tiles across
// u; the BF16 parts of the input tile with its halo live in LDS.

// LDS row stride of the input tile (BF16): the 80 values used, unpadded.  Measured
// with the LDS bank-conflict counter on the contrast workload: strides 88, 96, 104
// and 120 spend 49% of the kernel's LDS cycles in bank conflicts and a 16-byte XOR
// swizzle at stride 128 spends 32%; 80 spends none (head spread 12.0 -> 10.8 ms).
constexpr int kPsfStride = 80;
constexpr int kPsfRows = 64 + kPsfSplitMaxK - 1;

// B fragments: frag[((g * k + p) * 2 + part) * 64 + lane], part 0 = hi, 1 = lo.
__global__ __launch_bounds__(kBlock) void k_prep_psf_split(const float *__restrict__ ker, int G, int k,
                                                           uint4 *__restrict__ frag)
{
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= G * k * 2 * kWave) return;
    const int f = idx / kWave, lane = idx % kWave;
    const int part = f & 1, gp = f >> 1;
    const int q = lane >> 4, t = lane & 15;
    const int c = (k - 1) / 2;
    uint32_t h[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
        const int j = 8 * q + jj;
        const int col = t + c + 8 - j;
        const float v = (col >= 0 && col < k) ? ker[(int64_t)gp * k + col] : 0.0f;
        const uint32_t hi = bf16_rne(v);
        h[jj] = part ? bf16_rne(v - bf16_value(hi)) : hi;
    }
    frag[idx] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

__global__ __launch_bounds__(kBlock) void k_psf_split(const float *__restrict__ Y, int G, int nv, int nu, int k,
                                                      const uint4 *__restrict__ frag, float *__restrict__ out)
{
    __shared__ __align__(16) uint16_t th[kPsfRows * kPsfStride];
    __shared__ __align__(16) uint16_t tl[kPsfRows * kPsfStride];
    const int c = (k - 1) / 2;
    const int rows = 64 + k - 1;
    const int u0 = blockIdx.x * 64, v0 = blockIdx.y * 64, a = blockIdx.z;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int q = lane >> 4, r16 = lane & 15;
    const int64_t plane = (int64_t)nv * nu;
    floatx4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int g = 0; g < G; ++g) {
        const float *Yg = Y + ((int64_t)a * G + g) * plane;
        __syncthreads();
        // input tile: rows v0 - c .., columns u0 - 8 .. u0 + 71
        if ((nu & 3) == 0 && (reinterpret_cast<uintptr_t>(Y) & 15) == 0) {
            // whole 16-byte groups: a group is inside the detector or not at all
            for (int i = threadIdx.x; i < rows * 20; i += kBlock) {
                const int rr = i / 20, c4 = i - rr * 20;
                const int v = v0 - c + rr;
                const int u = u0 - 8 + 4 * c4;
                float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
                if (v >= 0 && v < nv && u >= 0 && u < nu)
                    y = *reinterpret_cast<const float4 *>(Yg + (int64_t)v * nu + u);
                uint32_t h01, l01, h23, l23;
                split_bf16x2(y.x, y.y, h01, l01);
                split_bf16x2(y.z, y.w, h23, l23);
                *reinterpret_cast<uint2 *>(th + rr * kPsfStride + 4 * c4) = make_uint2(h01, h23);
                *reinterpret_cast<uint2 *>(tl + rr * kPsfStride + 4 * c4) = make_uint2(l01, l23);
            }
        } else if (threadIdx.x < 240) {
            // thread t fills column pair t % 40 of rows t / 40, t / 40 + 6, ...
            const int col = 2 * (threadIdx.x % 40);
            const int u = u0 - 8 + col;
            const bool in0 = u >= 0 && u < nu, in1 = u + 1 >= 0 && u + 1 < nu;
            for (int rr = threadIdx.x / 40; rr < rows; rr += 6) {
                const int v = v0 - c + rr;
                const bool vin = v >= 0 && v < nv;
                const int64_t row = (int64_t)min(max(v, 0), nv - 1) * nu;
                const float y0 = (vin && in0) ? Yg[row + u] : 0.0f;
                const float y1 = (vin && in1) ? Yg[row + u + 1] : 0.0f;
                uint32_t hi, lo;
                split_bf16x2(y0, y1, hi, lo);
                *reinterpret_cast<uint32_t *>(th + rr * kPsfStride + col) = hi;
                *reinterpret_cast<uint32_t *>(tl + rr * kPsfStride + col) = lo;
            }
        }
        __syncthreads();
        const uint4 *fg = frag + (int64_t)g * k * 2 * kWave;
        for (int p = 0; p < k; ++p) {
            const bf16x8 bh = __builtin_bit_cast(bf16x8, fg[(2 * p) * kWave + lane]);
            const bf16x8 bl = __builtin_bit_cast(bf16x8, fg[(2 * p + 1) * kWave + lane]);
            const int row = 16 * wave + r16 - p + 2 * c;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int at = row * kPsfStride + 16 * ct + 8 * q;
                const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(th + at);
                const bf16x8 al = *reinterpret_cast<const bf16x8 *>(tl + at);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[ct], 0, 0, 0);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[ct], 0, 0, 0);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[ct], 0, 0, 0);
            }
        }
    }
    // D layout: lane (q, r16) holds rows 4q .. 4q + 3 of column r16
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int u = u0 + 16 * ct + r16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = v0 + 16 * wave + 4 * q + i;
            if (v < nv && u < nu) out[(int64_t)a * plane + (int64_t)v * nu + u] = acc[ct][i];
        }
    }
}

}  // namespace

hipError_t launch_prep_split(const float *mu, const SpecTables &t, const SplitTables &sp, uint4 *afrag,
                             float *wtile, hipStream_t stream)
{
    const int n = sp.T * sp.nkb * kWave;
    hipLaunchKernelGGL(k_prep_split, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, mu, t, sp, afrag,
                       wtile);
    return hipGetLastError();
}

#define FCAT_SPLIT_DISPATCH(MACRO) \
    if (t.mp == 8 && sp.nkb == 1) MACRO(8, 1) \
    else if (t.mp == 10 && sp.nkb == 1) MACRO(10, 1) \
    else if (t.mp == 12 && sp.nkb == 1) MACRO(12, 1) \
    else if (t.mp == 12 && sp.nkb == 2) MACRO(12, 2) \
    else if (t.mp == 16 && sp.nkb == 1) MACRO(16, 1) \
    else if (t.mp == 16 && sp.nkb == 2) MACRO(16, 2) \
    else if (t.mp == 32 && sp.nkb == 2) MACRO(32, 2) \
    else if (t.mp == 32 && sp.nkb == 3) MACRO(32, 3) \
    else return hipErrorInvalidValue;

hipError_t launch_project_rows_split(const TraceGeom &g, const int8_t *labels, const SpecTables &t,
                                     const SplitTables &sp, const float *flood, const float *scatter, int a0,
                                     int n_ang, float *Y, float *out, hipStream_t stream)
{
    (void)labels;
    const int64_t waves = (int64_t)n_ang * tiles_per_angle_host(g);
    const int nblk = padded_blocks(waves);
#define FCAT_LAUNCH_PR(MPV, NKBV)                                                                           \
    {                                                                                                       \
        hipLaunchKernelGGL((k_project_rows_split<MPV, NKBV>), dim3(nblk), dim3(kBlock), 0, stream, g, t, sp, \
                           flood, scatter, a0, n_ang, nblk, Y, out);                                   \
    }
    FCAT_SPLIT_DISPATCH(FCAT_LAUNCH_PR)
#undef FCAT_LAUNCH_PR
    return hipGetLastError();
}

hipError_t launch_prep_psf_split(const float *kernels, int G, int k, uint4 *frag, hipStream_t stream)
{
    if (k < 1 || k > kPsfSplitMaxK || (k & 1) == 0) return hipErrorInvalidValue;
    const int n = G * k * 2 * kWave;
    hipLaunchKernelGGL(k_prep_psf_split, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, kernels, G, k,
                       frag);
    return hipGetLastError();
}

hipError_t launch_psf_split(const float *Y, int n_ang, int G, int nv, int nu, int k, const uint4 *frag, float *out,
                            hipStream_t stream)
{
    if (k < 1 || k > kPsfSplitMaxK || (k & 1) == 0) return hipErrorInvalidValue;
    const dim3 grid((nu + 63) / 64, (nv + 63) / 64, n_ang);
    hipLaunchKernelGGL(k_psf_split, grid, dim3(kBlock), 0, stream, Y, G, nv, nu, k, frag, out);
    return hipGetLastError();
}

hipError_t launch_spectral_split(const float *L, int64_t n, const SpecTables &t, const SplitTables &sp,
                                 const float *i0, const float *S, float *Y, hipStream_t stream)
{
    const unsigned nblk = (unsigned)((n + kBlock - 1) / kBlock);
#define FCAT_LAUNCH_SP(MPV, NKBV)                                                                            \
    {                                                                                                        \
        hipLaunchKernelGGL((k_spectral_split<MPV, NKBV>), dim3(nblk), dim3(kBlock), 0, stream, L, n, t, sp, i0, \
                           S, Y);                                                                            \
    }
    FCAT_SPLIT_DISPATCH(FCAT_LAUNCH_SP)
#undef FCAT_LAUNCH_SP
    return hipGetLastError();
}

}  // namespace fcat
