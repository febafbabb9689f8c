// Learned surrogate of the primary spectral sum, on the gfx950 matrix cores.
//
// For a ray with path lengths L (Sec. II.F line integral over the labelled
// phantom of Sec. II.C) the primary part of Eq. 3 is
//     Yprim_g = sum_{e in g} w_e exp(-sum_m mu[m][e] L_m),   w_e = phi_e eta_e.
// The surrogate writes it as Yprim_g ~= W_g exp(-(sum_m lin[g][m] L_m + f(x)_g))
// with W_g = sum_{e in g} w_e, lin[g][m] = sum_{e in g} w_e mu[m][e] / W_g (the
// exact first-order term) and f = out_scale_g * MLP(x)_g, MLP a 64-64 SiLU
// perceptron of x_m = L_m in_scale_m, that learns the beam-hardening
// residual.
//
// Every product runs on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
// The forward pass (training and inference) splits each weight, input and
// hidden activation v into v_hi = bf16(v) and v_lo = bf16(v - v_hi) and forms
// a.b as a_hi.b_hi + a_lo.b_hi + a_hi.b_lo (the same three-term split as the
// L . mu contraction of the split-precision projector), so the network is
// evaluated to about FP32 accuracy rather than to BF16's 2^-9: the learned
// residual is of order one, and BF16 rounding alone would leave errors of
// order 1e-3 in the attenuation.  The backward pass uses the hi parts only
// (gradient directions need no more).  One wavefront handles 64 rays or
// samples; activations pass between layers through LDS.  Training writes one
// gradient partial per wavefront and the Adam kernel sums the partials in a
// fixed order, so training is deterministic.
#include "fcat_device.h"

namespace fcat {
namespace {

constexpr int H = FCAT_MLP_HIDDEN;     // 64
constexpr int SX = 40;                 // row stride (BF16) of 32-wide K buffers
constexpr int SH = 72;                 // row stride (BF16) of 64-wide K buffers
constexpr int SO = 17;                 // row stride (FP32) of the 16-wide output buffer

// Fragment index (in units of 64 lanes) of each weight view.  Lane
// (q = l/16, r = l%16) of tile t holds W[16 t + r][8 q + j], j < 8: the
// layout of the B operand of v_mfma_f32_16x16x32_bf16 for W[n][k] and,
// identically, of its A operand for W[m][k].
constexpr int kFragW1 = 0;     // [ht 0..3]          k < 16: W1_hi[n][k]; 16 <= k < 32: W1_hi[n][k - 16]
constexpr int kFragW1lo = 4;   // [ht 0..3]          k < 16: W1_lo[n][k]; else 0
constexpr int kFragW2 = 8;     // [ht 0..3][kb 0..1] W2_hi[n][32 kb + k]
constexpr int kFragW2lo = 16;  // [ht 0..3][kb 0..1] W2_lo
constexpr int kFragW3 = 24;    // [kb 0..1]          W3_hi[n][32 kb + k], n < n_out
constexpr int kFragW3lo = 26;  // [kb 0..1]          W3_lo
constexpr int kFragW3b = 28;   // [ht 0..3]          B[o][h2] = W3_hi[o][h2]   (dH2 = dZ3 W3)
constexpr int kFragW2b = 32;   // [ht 0..3][kb 0..1] B[h2][h1] = W2_hi[h2][h1] (dH1 = dZ2 W2)
// Inference views (see mlp_infer_wave): W1 scaled by log2(e) and W3 by
// 1/log2(e) before the hi/lo split, and the second- and third-layer weights
// listed over the hidden units in the order chained_unit gives.
constexpr int kFragW1i = 40;   // as kFragW1
constexpr int kFragW1iLo = 44; // as kFragW1lo
constexpr int kFragW3i = 48;   // [kb 0..1]          W3_hi[n][chained_unit(kb, q, j)] / log2(e), n < n_out
constexpr int kFragW3iLo = 50; // [kb 0..1]          lo part
constexpr int kFragW2c = 52;   // [ht 0..3][kb 0..1] W2_hi[16 ht + r][chained_unit(kb, q, j)]
constexpr int kFragW2cLo = 60; // [ht 0..3][kb 0..1] lo part
// The biases as the forward pass adds them, FP32: lane l holds entries
// 4 l .. 4 l + 3 of [log2(e) b1 (64) | log2(e) b2 (64) | b3 (n_out), zeros].
constexpr int kFragBias = 68;
constexpr int kBiasB2 = 64, kBiasB3 = 128;
static_assert(kFragBias + 1 == kMlpFrags, "fragment table size");
static_assert(kFragW1i == kMlpTrainFrags, "the training kernel reads the views before the inference views");
constexpr float kLog2e = 1.4426950408889634f;

// Hidden unit behind k index 8 q + j of the 32-wide block kb when a layer's
// accumulators feed the next layer in place: after a 16 x 16 x 32 product
// with the units as rows, lane (q, r) holds units 16 ht + 4 q + i (i < 4)
// of ray r, and block kb takes ht = 2 kb and 2 kb + 1.  A bijection of the
// 32 units of each block.
__device__ __host__ constexpr int chained_unit(int kb, int q, int j) { return 32 * kb + 16 * (j >> 2) + 4 * q + (j & 3); }

struct Offsets {
    int W1, b1, W2, b2, W3, b3, P;
};

__device__ __host__ inline Offsets param_offsets(int n_in, int n_out)
{
    Offsets o;
    o.W1 = 0;
    o.b1 = H * n_in;
    o.W2 = o.b1 + H;
    o.b2 = o.W2 + H * H;
    o.W3 = o.b2 + H;
    o.b3 = o.W3 + n_out * H;
    o.P = o.b3 + n_out;
    return o;
}

__device__ __forceinline__ bf16x8 frag_of(const uint4 *frag, int f, int lane)
{
    return __builtin_bit_cast(bf16x8, frag[f * kWave + lane]);
}

__device__ __forceinline__ bf16x8 lds_frag(const uint16_t *base, int stride, int row, int k)
{
    return *reinterpret_cast<const bf16x8 *>(base + row * stride + k);
}

// silu(z) = z sigmoid(z); sigmoid through v_exp_f32 and v_rcp_f32 (about
// 1 ulp each).  exp(-z) overflows to +inf for z < -88, and rcp(inf) = 0.
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }

__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

// Per-wavefront LDS of the forward pass: one 64-byte row per ray of the
// wavefront (4 KiB).  Row r first holds ray r's inputs [x_hi (16) | x_lo
// (16)] as four 16-byte chunks, chunk c at position c ^ ((r >> 2) & 3), so
// that the 16 rows one operand read touches fall on distinct banks.  Once
// its tile has been through the first layer, row r holds ray r's outputs,
// output o at word (o + (r >> 2)) & 15, so that 64 lanes reading the same
// output of their own rays fall on distinct banks.  The hidden activations
// never pass through LDS (see mlp_infer_wave).
constexpr int kInferRowBytes = 64;
constexpr int kInferLdsBytes = kWave * kInferRowBytes;

__device__ __forceinline__ int infer_chunk(int row, int c) { return row * kInferRowBytes + 16 * (c ^ ((row >> 2) & 3)); }
__device__ __forceinline__ int infer_out_word(int row, int o) { return row * (kInferRowBytes / 4) + ((o + (row >> 2)) & 15); }

// Output o of the ray of lane `lane`, after mlp_infer_wave.
__device__ __forceinline__ float mlp_out(const uint8_t *rows, int lane, int o)
{
    return reinterpret_cast<const float *>(rows)[infer_out_word(lane, o)];
}

// Bit ct set where any of lanes 16 ct .. 16 ct + 15 is set in a ballot.
__device__ __forceinline__ uint32_t tile_mask(uint64_t ballot)
{
    uint32_t t = 0;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) t |= ((ballot >> (16 * ct)) & 0xffffu) ? (1u << ct) : 0u;
    return t;
}

// With z' = log2(e) z, log2(e) silu(z) = z' / (1 + 2^-z'): one v_exp_f32,
// one add, one v_rcp_f32 and one multiply.
__device__ __forceinline__ float silu2(float zs)
{
    return zs * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-zs));
}

// SiLU of the 16 units a lane holds after one layer (acc[ht][i] = unit
// 16 ht + 4 q + i of its ray), split into hi/lo BF16 and packed as the next
// layer's B operands: block kb, element j = unit chained_unit(kb, q, j).
__device__ __forceinline__ void silu_pack(const floatx4 (&acc)[4], bf16x8 (&bh)[2], bf16x8 (&bl)[2])
{
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        uint32_t hi[4], lo[4];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const floatx4 &a = acc[2 * kb + t];
            split_bf16x2(silu2(a[0]), silu2(a[1]), hi[2 * t], lo[2 * t]);
            split_bf16x2(silu2(a[2]), silu2(a[3]), hi[2 * t + 1], lo[2 * t + 1]);
        }
        bh[kb] = __builtin_bit_cast(bf16x8, make_uint4(hi[0], hi[1], hi[2], hi[3]));
        bl[kb] = __builtin_bit_cast(bf16x8, make_uint4(lo[0], lo[1], lo[2], lo[3]));
    }
}

// Four consecutive entries of the bias fragment, from entry i (a multiple of 4).
__device__ __forceinline__ floatx4 bias4(const uint4 *frag, int i)
{
    return __builtin_bit_cast(floatx4, frag[kFragBias * kWave + i / 4]);
}

// Forward pass of the rays of the wavefront, one 16-ray tile (lanes
// 16 ct .. 16 ct + 15) at a time, tiles whose bit in `tiles` (one per 16
// lanes) is clear skipped.  The weights are the A operand (rows = units),
// the activations the B operand (columns = rays), so after each layer lane
// (q, r) holds units 16 ht + 4 q + i of ray r in its accumulators.  Those
// registers are the next layer's B operand as they stand: the hidden units
// are summed in the order chained_unit gives, and the second- and
// third-layer fragments list their weights in that order.  Only the
// inputs (to spread each ray's values over the four lane groups) and the
// outputs (to gather them back) pass through LDS.  The pass runs on
// z' = log2(e) z: W1 and b1, b2 carry the factor (W2 needs none, since the
// hidden values are log2(e) silu), and W3 its inverse, which yields the
// same network output as the unscaled form.  x: n_in values per lane, zero
// beyond; rows: this wavefront's kInferLdsBytes of LDS; the outputs are
// read back with mlp_out.
__device__ __forceinline__ void mlp_infer_wave(const float (&x)[16], const MlpTables &M, uint8_t *rows,
                                               uint32_t tiles = 0xfu)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane >> 4, r16 = lane & 15;
    {
        uint32_t hi[8], lo[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) split_bf16x2(x[2 * k], x[2 * k + 1], hi[k], lo[k]);
        *reinterpret_cast<uint4 *>(rows + infer_chunk(lane, 0)) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        *reinterpret_cast<uint4 *>(rows + infer_chunk(lane, 1)) = make_uint4(hi[4], hi[5], hi[6], hi[7]);
        *reinterpret_cast<uint4 *>(rows + infer_chunk(lane, 2)) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
        *reinterpret_cast<uint4 *>(rows + infer_chunk(lane, 3)) = make_uint4(lo[4], lo[5], lo[6], lo[7]);
    }
    wave_sync_lds();
#pragma unroll 1
    for (int ct = 0; ct < 4; ++ct) {
        if (!((tiles >> ct) & 1u)) continue;
        const int row = 16 * ct + r16;
        // a zero the compiler cannot see through, added to the fragment
        // table's address per tile: otherwise the table's loads are hoisted
        // out of the loop and their 112 registers held through it (and
        // through the walk it is fused with)
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        const uint4 *frag = M.frag + opaque;
        // layer 1: Z1 = W1_hi (x_hi + x_lo) + W1_lo x_hi + b1
        const bf16x8 bx = *reinterpret_cast<const bf16x8 *>(rows + infer_chunk(row, q));
        floatx4 acc[4];
#pragma unroll
        for (int ht = 0; ht < 4; ++ht) {
            acc[ht] = bias4(frag, 16 * ht + 4 * q);
            acc[ht] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_of(frag, kFragW1i + ht, lane), bx, acc[ht], 0, 0,
                                                              0);
            acc[ht] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_of(frag, kFragW1iLo + ht, lane), bx, acc[ht], 0,
                                                              0, 0);
        }
        bf16x8 hh[2], hl[2];
        silu_pack(acc, hh, hl);
        // layer 2: Z2 = W2_hi (H1_hi + H1_lo) + W2_lo H1_hi + b2
#pragma unroll
        for (int ht = 0; ht < 4; ++ht) {
            acc[ht] = bias4(frag, kBiasB2 + 16 * ht + 4 * q);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8 wh = frag_of(frag, kFragW2c + ht * 2 + kb, lane);
                acc[ht] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, hh[kb], acc[ht], 0, 0, 0);
                acc[ht] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, hl[kb], acc[ht], 0, 0, 0);
                acc[ht] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_of(frag, kFragW2cLo + ht * 2 + kb, lane),
                                                                  hh[kb], acc[ht], 0, 0, 0);
            }
        }
        silu_pack(acc, hh, hl);
        // layer 3: outputs 4 q .. 4 q + 3 of the tile's ray r16
        floatx4 o = bias4(frag, kBiasB3 + 4 * q);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 wh = frag_of(frag, kFragW3i + kb, lane);
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, hh[kb], o, 0, 0, 0);
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, hl[kb], o, 0, 0, 0);
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag_of(frag, kFragW3iLo + kb, lane), hh[kb], o, 0, 0, 0);
        }
        // row `row` has been read by this tile's first layer only: its words
        // now take the ray's outputs
        float *orow = reinterpret_cast<float *>(rows);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (4 * q + i < M.n_out) orow[infer_out_word(row, 4 * q + i)] = o[i];
    }
    wave_sync_lds();
}

// ------------------------------------------------------------ kernels

// Fragments of every weight view (FP32 master -> BF16 hi or lo part).
__device__ __forceinline__ float hi_part(float v) { return bf16_value(bf16_rne(v)); }

// The parameter whose BF16 hi (lo = false) or lo part fills element j of
// lane `lane` of training fragment f (f < kMlpTrainFrags), or -1 for a zero
// element; the same views k_mlp_prep builds.
__device__ int train_frag_source(int f, int lane, int j, int n_in, int n_out, bool &lo)
{
    const Offsets off = param_offsets(n_in, n_out);
    const int q = lane >> 4, r16 = lane & 15, kk = 8 * q + j;
    lo = false;
    if (f < kFragW1lo) {                        // [W1_hi | W1_hi]
        const int n = 16 * (f - kFragW1) + r16, k = kk & 15;
        return k < n_in ? off.W1 + n * n_in + k : -1;
    }
    if (f < kFragW2) {                          // [W1_lo | 0]
        lo = true;
        const int n = 16 * (f - kFragW1lo) + r16;
        return kk < n_in ? off.W1 + n * n_in + kk : -1;
    }
    if (f < kFragW3) {                          // W2_hi, W2_lo
        lo = f >= kFragW2lo;
        const int t = f - (lo ? kFragW2lo : kFragW2);
        return off.W2 + (16 * (t / 2) + r16) * H + 32 * (t % 2) + kk;
    }
    if (f < kFragW3b) {                         // W3_hi, W3_lo
        lo = f >= kFragW3lo;
        const int kb = f - (lo ? kFragW3lo : kFragW3);
        return r16 < n_out ? off.W3 + r16 * H + 32 * kb + kk : -1;
    }
    if (f < kFragW2b)                           // B[k = o][n = h2] = W3[o][h2]
        return kk < n_out ? off.W3 + kk * H + 16 * (f - kFragW3b) + r16 : -1;
    const int ct = (f - kFragW2b) / 2, kb = (f - kFragW2b) % 2;   // B[k = h2][n = h1] = W2[h2][h1]
    return off.W2 + (32 * kb + kk) * H + 16 * ct + r16;
}

// Inverse of train_frag_source: for each parameter p, the BF16 elements of
// the training fragments that hold a part of it, inv[kMlpViews p + i] =
// element index (fragment f, lane, j: (64 f + lane) 8 + j) | lo << 31 for
// i < cnt[p]; cnt [P] must start at zero.  Every parameter fills at
// most three elements (a W1 weight its hi part twice and its lo part once,
// a W2 or W3 weight its hi and lo parts and one transposed hi part).
__global__ __launch_bounds__(kBlock) void k_mlp_frag_inverse(int n_in, int n_out, int *__restrict__ cnt,
                                                            uint32_t *__restrict__ inv)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= kMlpTrainFrags * kWave * 8) return;
    bool lo;
    const int p = train_frag_source(s / (8 * kWave), (s / 8) % kWave, s % 8, n_in, n_out, lo);
    if (p < 0) return;
    const int i = atomicAdd(cnt + p, 1);
    if (i < kMlpViews) inv[kMlpViews * p + i] = (uint32_t)s | (lo ? 0x80000000u : 0u);
}

__global__ __launch_bounds__(kBlock) void k_mlp_prep(const float *__restrict__ params, int n_in, int n_out,
                                                     uint4 *__restrict__ frag, int n_frags)
{
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n_frags * kWave) return;
    const int fi = idx / kWave, lane = idx % kWave;
    const int q = lane >> 4, r16 = lane & 15;
    const Offsets off = param_offsets(n_in, n_out);
    if (fi == kFragBias) {
        float b[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = 4 * lane + c;
            b[c] = i < kBiasB2 ? kLog2e * params[off.b1 + i]
                 : i < kBiasB3 ? kLog2e * params[off.b2 + i - kBiasB2]
                 : i < kBiasB3 + n_out ? params[off.b3 + i - kBiasB3] : 0.0f;
        }
        frag[idx] = make_uint4(__float_as_uint(b[0]), __float_as_uint(b[1]), __float_as_uint(b[2]),
                               __float_as_uint(b[3]));
        return;
    }
    // the first-layer inference views are the W1 views of scaled weights
    int f = fi;
    float scale = 1.0f;
    if (fi >= kFragW1i && fi < kFragW3i) {
        f = kFragW1 + (fi - kFragW1i);
        scale = kLog2e;
    }
    uint32_t h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int kk = 8 * q + j;
        float v = 0.0f;
        if (f >= kFragW2c) {                     // W2 in chained order, hi or lo
            const bool lo = f >= kFragW2cLo;
            const int t = f - (lo ? kFragW2cLo : kFragW2c);
            const float w = params[off.W2 + (16 * (t / 2) + r16) * H + chained_unit(t % 2, q, j)];
            v = lo ? w - hi_part(w) : w;
        } else if (f >= kFragW3i) {              // W3 / log2(e) in chained order, hi or lo
            const bool lo = f >= kFragW3iLo;
            const int kb = f - (lo ? kFragW3iLo : kFragW3i);
            if (r16 < n_out) {
                const float w = (1.0f / kLog2e) * params[off.W3 + r16 * H + chained_unit(kb, q, j)];
                v = lo ? w - hi_part(w) : w;
            }
        } else if (f < kFragW1lo) {                     // [W1_hi | W1_hi]
            const int n = 16 * (f - kFragW1) + r16, k = kk & 15;
            if (k < n_in) v = hi_part(scale * params[off.W1 + n * n_in + k]);
        } else if (f < kFragW2) {                // [W1_lo | 0]
            const int n = 16 * (f - kFragW1lo) + r16;
            if (kk < n_in) {
                const float w = scale * params[off.W1 + n * n_in + kk];
                v = w - hi_part(w);
            }
        } else if (f < kFragW3) {                // W2_hi, W2_lo
            const bool lo = f >= kFragW2lo;
            const int t = f - (lo ? kFragW2lo : kFragW2);
            const int n = 16 * (t / 2) + r16, k = 32 * (t % 2) + kk;
            const float w = params[off.W2 + n * H + k];
            v = lo ? w - hi_part(w) : w;
        } else if (f < kFragW3b) {               // W3_hi, W3_lo
            const bool lo = f >= kFragW3lo;
            const int kb = f - (lo ? kFragW3lo : kFragW3);
            const int n = r16, k = 32 * kb + kk;
            if (n < n_out) {
                const float w = scale * params[off.W3 + n * H + k];
                v = lo ? w - hi_part(w) : w;
            }
        } else if (f < kFragW2b) {               // B[k = o][n = h2] = W3[o][h2]
            const int n = 16 * (f - kFragW3b) + r16;
            if (kk < n_out) v = params[off.W3 + kk * H + n];
        } else {                                 // B[k = h2][n = h1] = W2[h2][h1]
            const int ct = (f - kFragW2b) / 2, kb = (f - kFragW2b) % 2;
            const int n = 16 * ct + r16, k = 32 * kb + kk;
            v = params[off.W2 + k * H + n];
        }
        h[j] = bf16_rne(v);
    }
    frag[idx] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// lin[g][m] = sum_{e in g} w_e mu[m][e] / W_g
__global__ __launch_bounds__(kBlock) void k_mlp_linear(const float *__restrict__ mu, SpecTables T,
                                                       float *__restrict__ lin)
{
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= T.G * T.M) return;
    const int g = idx / T.M, m = idx % T.M;
    double a = 0.0, b = 0.0;
    for (int e = T.gstart[g]; e < T.gstart[g + 1]; ++e) {
        a += (double)T.w[e] * (double)mu[(int64_t)m * T.E + e];
        b += (double)T.w[e];
    }
    lin[idx] = (float)(a / b);
}

// Validation cell of a hit ray: the dominant material by optical depth
// mbar_m L_m, times 16 bins of the total optical depth over
// [cell_lo, cell_hi); -1 outside the training range (some x_m > 1 or the
// depth outside the bins).
__device__ __forceinline__ int cell_of(const float (&L)[16], const float (&x)[16], const MlpTables &M)
{
    bool inside = true;
    int dom = 0;
    float best = -1.0f, tau = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        if (m < M.n_in) {
            inside = inside && x[m] <= 1.0f;
            const float t = __fmul_rn(M.mbar[m], L[m]);    // no contraction: the cell is an integer decision
            tau = __fadd_rn(tau, t);
            if (t > best) {
                best = t;
                dom = m;
            }
        }
    }
    const float b = floorf(__fdiv_rn(__fmul_rn((float)FCAT_MLP_CELLS, __fsub_rn(tau, M.cell_lo)),
                                     __fsub_rn(M.cell_hi, M.cell_lo)));
    if (!inside || !(b >= 0.0f && b < (float)FCAT_MLP_CELLS)) return -1;
    return dom * FCAT_MLP_CELLS + (int)b;
}

__device__ __forceinline__ bool in_domain(const float (&L)[16], const float (&x)[16], const MlpTables &M)
{
    const int c = cell_of(L, x, M);
    return c >= 0 && M.cell_ok[c] != 0;
}

// Spectral stage with the surrogate: L [n][M] in, group signals out.
template <int MP>
__global__ __launch_bounds__(kBlock) void k_mlp_spectral(SpecTables T, MlpTables M, SurrogateIO io)
{
    __shared__ __align__(16) uint8_t lds[(kBlock / kWave) * kInferLdsBytes];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    uint8_t *rows = lds + wave * kInferLdsBytes;
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < io.n;
    float L[16], x[16];
    float tot = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        L[m] = (valid && m < T.M) ? io.L[r * T.M + m] : 0.0f;
        x[m] = m < M.n_in ? __fmul_rn(L[m], M.in_scale[m]) : 0.0f;
        tot += L[m];
    }
    const bool hit = valid && tot > 0.0f;
    const bool use = hit && (io.force_mlp || in_domain(L, x, M));
    const uint64_t use_mask = __ballot(use);
    if (use_mask != 0) mlp_infer_wave(x, M, rows, tile_mask(use_mask));
    if (io.counts && valid) {
        const uint64_t bu = __ballot(use), bh = __ballot(hit);
        if (lane == 0) {
            atomicAdd(io.counts + 0, (int)__popcll(bu));
            atomicAdd(io.counts + 1, (int)__popcll(bh & ~bu));
        }
    }
    if (!valid) return;
    float Lp[MP];
#pragma unroll
    for (int m = 0; m < MP; ++m) Lp[m] = m < 16 ? L[m] : 0.0f;
    const int64_t al = r / io.plane, pix = r - al * io.plane;
    const float i0 = io.flood ? io.flood[pix] : 1.0f;
    const float sc = io.scatter ? io.scatter[r] : 0.0f;
    float total = 0.0f;
    for (int g = 0; g < T.G; ++g) {
        float prim;
        if (use) {
            float z = M.out_scale[g] * mlp_out(rows, lane, g);
#pragma unroll
            for (int m = 0; m < 16; ++m)
                if (m < T.M) z = fmaf(M.lin[g * T.M + m], L[m], z);
            prim = T.Wg[g] * expf(-z);
        } else if (hit) {
            prim = group_sum<MP>(Lp, T, T.gstart[g], T.gstart[g + 1]);
        } else {
            prim = T.Wg[g];
        }
        const float y = fmaf(i0, prim, T.Wsg[g] * sc);
        if (io.Y)
            io.Y[(al * T.G + g) * io.plane + pix] = y;
        else
            total += y;
    }
    if (io.out) io.out[r] = total;
    flag_nonfinite(io.bad, i0, sc);
}

// The surrogate projector in one pass: the walk of k_project_rows, then,
// for the wavefronts whose rays all lie in cells the held-out validation
// accepted, the network on the matrix cores, and the exact spectral sum for
// the rest; scatter and group signals as in k_project_rows.  The path lengths stay in registers.
// The walk's LDS block of each wavefront is reused for the network's
// input/output rows once the walk is done, so the network needs no LDS of
// its own; its weights are read from the fragment table (L2-resident,
// 69 KiB), since LDS for a copy per workgroup would cap the walk at four
// wavefronts per SIMD.
template <int MP>
constexpr int fused_wave_floats()
{
    constexpr int a = (mat_acc_floats<MP>() + 3) / 4 * 4;
    return a > kInferLdsBytes / 4 ? a : kInferLdsBytes / 4;
}

// Occupancy the fused kernel is compiled to: what the walk's LDS block
// allows, at most 6 wavefronts per SIMD.  On the head workload with every
// hit ray on the network the kernel took 89.7 ms at 8 (64 registers, a few
// values spilled around the network), 87.9 at 6, 99.7 at 5 and 111.5 at 4
// (the plain walk: 66.3): the network's fragment loads wait on L2 one or two
// at a time whatever the register budget, and more wavefronts hide that.
template <int MP>
constexpr int fused_waves_per_simd()
{
    constexpr int per_cu = (160 * 1024) / ((kBlock / kWave) * fused_wave_floats<MP>() * 4) * (kBlock / kWave);
    return per_cu / 4 < 6 ? per_cu / 4 : 6;
}

template <int MP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(fused_waves_per_simd<MP>())))
void k_project_rows_mlp(TraceGeom G, SpecTables T, MlpTables M,
                                                             const float *__restrict__ flood,
                                                             const float *__restrict__ scatter, int a0, int n_ang,
                                                             int nblk_pad, float *__restrict__ Y,
                                                             float *__restrict__ out, int *__restrict__ slots)
{
    __shared__ __align__(16) float lds_all[(kBlock / kWave) * fused_wave_floats<MP>()];
    const int blk = xcd_block(nblk_pad);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = blk * (kBlock / kWave) + wave;
    if (gw >= n_ang * tiles_per_angle(G)) return;
    const PixelOf px = pixel_of(G, gw, lane);
    const int al = px.al, iv = px.iv, iu = px.iu;
    const int a = a0 + al;
    const bool valid = px.valid;
    float *block = lds_all + wave * fused_wave_floats<MP>();

    double st, ct;
    // evaluated per lane: reading the projector's per-angle table here (as the
    // plain walk does) measured slower in this kernel, 86 against 81 ms
    sincos(angle_of(G, a), &st, &ct);
    float L[MP];
    Ray r{};
    const bool hit = valid && setup_ray(G, ct, st, iv, iu, r);
    trace_bricks<MP>(r, hit, G, G.labels_bm, G.bricks, block, L);

    float L16[16], x[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        L16[m] = m < MP ? L[m] : 0.0f;
        x[m] = m < M.n_in ? __fmul_rn(L16[m], M.in_scale[m]) : 0.0f;
    }
    // The network is taken wavefront by wavefront: only where every ray of
    // the wavefront that meets the phantom lies in a validated cell.  A
    // wavefront with one ray outside them takes the exact sum for all its
    // rays (never less accurate), since its lanes run in lockstep and would
    // otherwise pay for both the network and the exact sum.
    // (both ballots run in every lane: inside a short-circuit && the second
    // would see only the lanes already accepted)
    const bool ok = hit && in_domain(L16, x, M);
    const uint64_t outside = __ballot(hit && !ok);
    const bool use = ok && outside == 0;
    const uint64_t use_mask = __ballot(use);
    uint8_t *rows = reinterpret_cast<uint8_t *>(block);
    if (use_mask != 0) {
        wave_sync_lds();      // the walk's sums have been read: the block becomes the network's rows
        mlp_infer_wave(x, M, rows, tile_mask(use_mask));
    }
    const uint64_t hit_mask = __ballot(hit), valid_mask = __ballot(valid);
    if (!valid) return;

    const int64_t plane = (int64_t)G.nu * G.nv;
    const int64_t pix = (int64_t)iv * G.nu + iu;
    const float i0 = flood ? flood[pix] : 1.0f;
    const float sc = scatter ? scatter[(int64_t)a * plane + pix] : 0.0f;
    float total = 0.0f;
    const auto *Wg = const_table(T.Wg), *Wsg = const_table(T.Wsg);
    const auto *lin = const_table(M.lin), *out_scale = const_table(M.out_scale);
    auto emit = [&](int g, float prim) {
        const float y = fmaf(i0, prim, Wsg[g] * sc);
        if (Y)
            Y[((int64_t)al * T.G + g) * plane + pix] = y;
        else
            total += y;
    };
    // Two loops on a wavefront-uniform choice; the exact one is the plain
    // projector's.
    if (use_mask != 0) {
        for (int g = 0; g < T.G; ++g) {
            float prim = Wg[g];
            if (use) {
                float z = out_scale[g] * mlp_out(rows, lane, g);
#pragma unroll
                for (int m = 0; m < MP; ++m)
                    if (m < T.M) z = fmaf(lin[g * T.M + m], L[m], z);
                prim *= expf(-z);
            }
            emit(g, prim);
        }
    } else {
        const bool any_hit = hit_mask != 0;
        for (int g = 0; g < T.G; ++g)
            emit(g, any_hit ? group_sum<MP>(L, T, T.gstart[g], T.gstart[g + 1]) : Wg[g]);
    }
    if (!Y) out[(int64_t)a * plane + pix] = total;
    // after the last table read, as flag_nonfinite: a store before them would
    // turn the tables' wave-uniform scalar loads into per-lane vector loads
    if (slots && lane == __ffsll((unsigned long long)valid_mask) - 1) {
        int *slot = slots + (gw % kCountSlots) * kCountSlotInts;
        atomicAdd(slot + 0, (int)__popcll(use_mask));
        atomicAdd(slot + 1, (int)__popcll(hit_mask & ~use_mask));
    }
    flag_nonfinite(G.bad, i0, sc);
}

// Totals of the count slots (see kCountSlots), added to counts[0] and counts[1].
__global__ __launch_bounds__(kCountSlots) void k_count_slots_sum(const int *__restrict__ slots,
                                                                 int *__restrict__ counts)
{
    __shared__ int part[2][kCountSlots / kWave];
    const int t = threadIdx.x;
    int a = slots[t * kCountSlotInts + 0], b = slots[t * kCountSlotInts + 1];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_down(a, off);
        b += __shfl_down(b, off);
    }
    if ((t & (kWave - 1)) == 0) {
        part[0][t / kWave] = a;
        part[1][t / kWave] = b;
    }
    __syncthreads();
    if (t == 0) {
        int sa = 0, sb = 0;
        for (int w = 0; w < kCountSlots / kWave; ++w) {
            sa += part[0][w];
            sb += part[1][w];
        }
        atomicAdd(counts + 0, sa);
        atomicAdd(counts + 1, sb);
    }
}

struct TrainLds {
    uint16_t X[kWave * SX];      // inputs, later dZ3 [sample][o]
    uint16_t XT[16 * SH];        // inputs transposed [m][sample]
    uint16_t H1[kWave * SH];     // layer-1 activations, later dZ2 [sample][h2]
    uint16_t H1T[kWave * SH];    // [h1][sample]
    uint16_t H2[kWave * SH];     // layer-2 activations, later dZ2T [h2][sample]
    uint16_t H2T[kWave * SH];    // [h2][sample]
    uint16_t D3T[16 * SH];       // dZ3 transposed [o][sample]
    uint16_t D1T[kWave * SH];    // dZ1 transposed [h1][sample]
    float Tg[kWave * SO];        // residual targets [sample][o]
    float Wt[kWave * SO];        // loss weights [sample][o]
};

// Forward + backward of one 64-sample tile per workgroup of four wavefronts.
// Samples order[base + i], i < count; the loss is the mean over `count`
// samples and n_out outputs of omega (s f - r)^2, with r the residual
// target, s = out_scale and omega = min(1, Y_g / (1e-3 sum_g Y_g))^2.  Writes
// the gradient partial of the tile to partial[blockIdx.x][P] and its loss
// sum to loss_partial[blockIdx.x].
//
// Wavefront w takes the tile's samples 16 w .. 16 w + 15 (row tile w of
// every sample-major array) through the three layers and back; the
// weight gradients, which sum over all 64 samples, are then split by output
// tile: wavefront w forms tile w of dW3, row tile w of dW2 and of dW1, with
// the same products in the same order as over the whole tile.  The four
// wavefronts' bias and loss sums are added in wavefront order, so training
// stays deterministic.
constexpr int kGradWaves = 4;
__global__ __launch_bounds__(kGradWaves * kWave) void k_mlp_grad(SpecTables T, MlpTables M, const float *__restrict__ Lin,
                                                                 const float *__restrict__ Yin, int64_t n_all,
                                                                 const int32_t *__restrict__ order, int64_t base,
                                                                 int count, float *__restrict__ partial,
                                                                 float *__restrict__ loss_partial)
{
    __shared__ __align__(16) TrainLds S;
    constexpr int kRedB2 = 64, kRedB3 = 128, kRedLoss = 144;
    __shared__ float red[kGradWaves][kRedLoss + 1];   // per wavefront: db1 [64], db2 [64], db3 [16], loss
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane >> 4, r16 = lane & 15;
    const int rt = wave;                 // this wavefront's row tile of samples
    const Offsets off = param_offsets(M.n_in, M.n_out);
    const float *P = M.params;
    const int n_in = M.n_in, n_out = M.n_out;
    const float inv_n = 1.0f / ((float)count * (float)n_out);

    if (wave == 0) {
        // inputs and residual targets r_g = -ln(Y_g / W_g) - sum_m lin[g][m] L_m,
        // one sample per lane
        const int local = blockIdx.x * kWave + lane;
        const bool valid = local < count;
        const int64_t s = valid ? (int64_t)(order ? order[base + local] : base + local) : 0;
        float L[16], x[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            L[m] = (valid && m < n_in) ? Lin[s * n_in + m] : 0.0f;
            x[m] = m < n_in ? L[m] * M.in_scale[m] : 0.0f;
        }
        float ysum = 0.0f;
        for (int g = 0; g < n_out; ++g) ysum += valid ? Yin[(int64_t)g * n_all + s] : 0.0f;
        for (int g = 0; g < 16; ++g) {
            float t = 0.0f, om = 0.0f;
            if (valid && g < n_out) {
                const float y = Yin[(int64_t)g * n_all + s];
                const float f = fminf(1.0f, y / (kMlpShareFloor * ysum));
                if (f > 0.0f) {                    // y > 0: the target is finite
                    t = -logf(y / T.Wg[g]);
#pragma unroll
                    for (int m = 0; m < 16; ++m)
                        if (m < n_in) t -= M.lin[g * n_in + m] * L[m];
                    om = f * f;
                }
            }
            S.Tg[lane * SO + g] = t;
            S.Wt[lane * SO + g] = om;
        }
        // row = [x_hi (16) | x_lo (16)]; the transpose keeps x_hi for dW1
        uint32_t hi[8], lo[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) split_bf16x2(x[2 * k], x[2 * k + 1], hi[k], lo[k]);
        uint4 *row = reinterpret_cast<uint4 *>(S.X + lane * SX);
        row[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        row[1] = make_uint4(hi[4], hi[5], hi[6], hi[7]);
        row[2] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
        row[3] = make_uint4(lo[4], lo[5], lo[6], lo[7]);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            S.XT[(2 * k) * SH + lane] = (uint16_t)(hi[k] & 0xffffu);
            S.XT[(2 * k + 1) * SH + lane] = (uint16_t)(hi[k] >> 16);
        }
    }
    __syncthreads();
    uint16_t *const Hlo = S.D1T;     // lo parts of H1, then of H2 (D1T is free until the backward pass)

    // ---- forward, samples of row tile rt
    floatx4 Z1[4], Z2[4], acc[4];
    {
        const bf16x8 a = lds_frag(S.X, SX, 16 * rt + r16, 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            Z1[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW1 + ct, lane),
                                                             floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            Z1[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW1lo + ct, lane), Z1[ct], 0, 0, 0);
        }
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const float b = P[off.b1 + 16 * ct + r16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Z1[ct][i] += b;
            const float hv = silu(Z1[ct][i]);
            const uint32_t hb = bf16_rne(hv);
            const uint16_t h = (uint16_t)hb;
            const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
            S.H1[row * SH + col] = h;
            S.H1T[col * SH + row] = h;
            Hlo[row * SH + col] = (uint16_t)bf16_rne(hv - bf16_value(hb));
        }
    }
    wave_sync_lds();
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) Z2[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 a = lds_frag(S.H1, SH, 16 * rt + r16, 32 * kb + 8 * q);
        const bf16x8 al = lds_frag(Hlo, SH, 16 * rt + r16, 32 * kb + 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const bf16x8 wh = frag_of(M.frag, kFragW2 + ct * 2 + kb, lane);
            Z2[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wh, Z2[ct], 0, 0, 0);
            Z2[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, wh, Z2[ct], 0, 0, 0);
            Z2[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW2lo + ct * 2 + kb, lane), Z2[ct],
                                                             0, 0, 0);
        }
    }
    wave_sync_lds();
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const float b = P[off.b2 + 16 * ct + r16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Z2[ct][i] += b;
            const float hv = silu(Z2[ct][i]);
            const uint32_t hb = bf16_rne(hv);
            const uint16_t h = (uint16_t)hb;
            const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
            S.H2[row * SH + col] = h;
            S.H2T[col * SH + row] = h;
            Hlo[row * SH + col] = (uint16_t)bf16_rne(hv - bf16_value(hb));
        }
    }
    wave_sync_lds();
    floatx4 o3 = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 a = lds_frag(S.H2, SH, 16 * rt + r16, 32 * kb + 8 * q);
        const bf16x8 al = lds_frag(Hlo, SH, 16 * rt + r16, 32 * kb + 8 * q);
        const bf16x8 wh = frag_of(M.frag, kFragW3 + kb, lane);
        o3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wh, o3, 0, 0, 0);
        o3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, wh, o3, 0, 0, 0);
        o3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW3lo + kb, lane), o3, 0, 0, 0);
    }
    wave_sync_lds();

    // ---- output error dZ3 = 2 omega (s f - r) s / (count n_out)
    const float b3 = r16 < n_out ? P[off.b3 + r16] : 0.0f;
    const float osc = r16 < n_out ? M.out_scale[r16] : 0.0f;
    float lsum = 0.0f, db3 = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = 16 * rt + 4 * q + i;
        const bool live = r16 < n_out && (int)(blockIdx.x * kWave + row) < count;
        const float om = live ? S.Wt[row * SO + r16] : 0.0f;
        const float d = live ? osc * (o3[i] + b3) - S.Tg[row * SO + r16] : 0.0f;
        lsum += om * d * d;
        const float g = 2.0f * om * d * osc * inv_n;
        db3 += g;
        const uint16_t gb = (uint16_t)bf16_rne(g);
        S.X[row * SX + r16] = gb;            // dZ3 [sample][o], o < 16
        S.X[row * SX + 16 + r16] = 0;        // K padding up to 32
        S.D3T[r16 * SH + row] = gb;          // dZ3 transposed [o][sample]
    }
    wave_sync_lds();

    // ---- dH2 = dZ3 W3 ; dZ2 = dH2 * silu'(Z2)
    {
        const bf16x8 a = lds_frag(S.X, SX, 16 * rt + r16, 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW3b + ct, lane),
                                                              floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
    // H2 (read by every wavefront's third layer) and the lo parts are
    // overwritten below by other wavefronts' samples: all must be past it
    __syncthreads();
    float db2[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float g = acc[ct][i] * dsilu(Z2[ct][i]);
            db2[ct] += g;
            const uint16_t gb = (uint16_t)bf16_rne(g);
            const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
            S.H1[row * SH + col] = gb;       // dZ2 [sample][h2]
            S.H2[col * SH + row] = gb;       // dZ2 transposed [h2][sample]
        }
    wave_sync_lds();

    // ---- dH1 = dZ2 W2 ; dZ1 = dH1 * silu'(Z1)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 a = lds_frag(S.H1, SH, 16 * rt + r16, 32 * kb + 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW2b + ct * 2 + kb, lane), acc[ct],
                                                              0, 0, 0);
    }
    float db1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float g = acc[ct][i] * dsilu(Z1[ct][i]);
            db1[ct] += g;
            const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
            S.D1T[col * SH + row] = (uint16_t)bf16_rne(g);   // dZ1 transposed [h1][sample]
        }
    // bias and loss sums of this wavefront's samples (reduce the 4 lane quarters)
    db3 += __shfl_xor(db3, 16);
    db3 += __shfl_xor(db3, 32);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        db2[ct] += __shfl_xor(db2[ct], 16);
        db2[ct] += __shfl_xor(db2[ct], 32);
        db1[ct] += __shfl_xor(db1[ct], 16);
        db1[ct] += __shfl_xor(db1[ct], 32);
    }
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) lsum += __shfl_xor(lsum, sh);
    if (q == 0) {
        red[wave][kRedB3 + r16] = db3;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            red[wave][kRedB2 + 16 * ct + r16] = db2[ct];
            red[wave][16 * ct + r16] = db1[ct];
        }
    }
    if (lane == 0) red[wave][kRedLoss] = lsum;
    __syncthreads();

    float *out = partial + (int64_t)blockIdx.x * off.P;
    // ---- dW3[o][h2] = sum_s dZ3[s][o] H2[s][h2], output tile ct = wave
    {
        const int ct = wave;
        floatx4 w3 = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            w3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_frag(S.D3T, SH, r16, 32 * kb + 8 * q),
                                                         lds_frag(S.H2T, SH, 16 * ct + r16, 32 * kb + 8 * q), w3, 0, 0,
                                                         0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 4 * q + i;
            if (o < n_out) out[off.W3 + o * H + 16 * ct + r16] = w3[i];
        }
    }
    // ---- dW2[h2][h1] = sum_s dZ2[s][h2] H1[s][h1], row tile rt = wave
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 a = lds_frag(S.H2, SH, 16 * rt + r16, 32 * kb + 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, lds_frag(S.H1T, SH, 16 * ct + r16, 32 * kb + 8 * q),
                                                              acc[ct], 0, 0, 0);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[off.W2 + (16 * rt + 4 * q + i) * H + 16 * ct + r16] = acc[ct][i];
    // ---- dW1[h1][m] = sum_s dZ1[s][h1] X[s][m], row tile rt = wave
    {
        floatx4 w1 = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            w1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_frag(S.D1T, SH, 16 * rt + r16, 32 * kb + 8 * q),
                                                         lds_frag(S.XT, SH, r16, 32 * kb + 8 * q), w1, 0, 0, 0);
        if (r16 < n_in) {
#pragma unroll
            for (int i = 0; i < 4; ++i) out[off.W1 + (16 * rt + 4 * q + i) * n_in + r16] = w1[i];
        }
    }
    // ---- biases and loss: the wavefronts' sums in wavefront order
    if (wave == 0) {
        const float s1 = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        const float s2 = ((red[0][kRedB2 + lane] + red[1][kRedB2 + lane]) + red[2][kRedB2 + lane]) + red[3][kRedB2 + lane];
        out[off.b1 + lane] = s1;
        out[off.b2 + lane] = s2;
        if (lane < n_out)
            out[off.b3 + lane] =
                ((red[0][kRedB3 + lane] + red[1][kRedB3 + lane]) + red[2][kRedB3 + lane]) + red[3][kRedB3 + lane];
        if (lane == 0)
            loss_partial[blockIdx.x] =
                ((red[0][kRedLoss] + red[1][kRedLoss]) + red[2][kRedLoss]) + red[3][kRedLoss];
    }
}

// grad[p] = sum over the gradient partials, in a fixed order: wavefront i
// of a workgroup sums partials i, i + 4, i + 8, ... of the workgroup's 64
// parameters (coalesced rows), then the four sums are added in wavefront
// order.  Deterministic, and spread over P / 64 workgroups with chains a
// quarter as long as one sum per parameter.  Where params is given, the
// Adam update (Kingma & Ba 2015, Algorithm 1) with bias correction for step
// t follows; loss_out (if given) receives sum_w loss_partial[w] * loss_scale.
constexpr int kReduceWaves = kBlock / kWave;
__global__ __launch_bounds__(kBlock) void k_mlp_reduce_adam(const float *__restrict__ partial, int nparts, int P,
                                                            float *__restrict__ grad, float *__restrict__ params,
                                                            float *__restrict__ m, float *__restrict__ v, int step,
                                                            float lr, float beta1, float beta2, float eps,
                                                            const float *__restrict__ loss_partial, float loss_scale,
                                                            float *__restrict__ loss_out, const int *__restrict__ cnt,
                                                            const uint32_t *__restrict__ inv,
                                                            uint16_t *__restrict__ frag16)
{
    __shared__ float sums[kReduceWaves][kWave];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int p = blockIdx.x * kWave + lane;
    float g = 0.0f;
    if (p < P)
        for (int w = wave; w < nparts; w += kReduceWaves) g += partial[(int64_t)w * P + p];
    sums[wave][lane] = g;
    __syncthreads();
    if (wave != 0) return;
    if (blockIdx.x == 0 && lane == 0 && loss_out) {
        float l = 0.0f;
        for (int w = 0; w < nparts; ++w) l += loss_partial[w];
        *loss_out = l * loss_scale;
    }
    if (p >= P) return;
    g = (sums[0][lane] + sums[1][lane]) + (sums[2][lane] + sums[3][lane]);
    if (grad) grad[p] = g;
    if (params) {
        const float mt = beta1 * m[p] + (1.0f - beta1) * g;
        const float vt = beta2 * v[p] + (1.0f - beta2) * g * g;
        m[p] = mt;
        v[p] = vt;
        const float mhat = mt / (1.0f - powf(beta1, (float)step));
        const float vhat = vt / (1.0f - powf(beta2, (float)step));
        const float w = params[p] - lr * mhat / (sqrtf(vhat) + eps);
        params[p] = w;
        if (inv) {
            // the next step's training fragments: this parameter's BF16 parts,
            // as k_mlp_prep would build them from w
            const int n = min(cnt[p], kMlpViews);
            for (int i = 0; i < n; ++i) {
                const uint32_t e = inv[kMlpViews * p + i];
                frag16[e & 0x7fffffffu] = (uint16_t)((e >> 31) ? bf16_rne(w - hi_part(w)) : bf16_rne(w));
            }
        }
    }
}

// Held-out validation: per ray, the largest relative error over groups of
// the predicted primary signal, with a floor of 1e-3 of the ray's total
// signal; its maximum and the sample count per cell.
__global__ __launch_bounds__(kBlock) void k_mlp_validate(SpecTables T, MlpTables M, const float *__restrict__ Lin,
                                                         const float *__restrict__ Yin, int64_t n,
                                                         unsigned *__restrict__ cell_err_bits,
                                                         int *__restrict__ cell_count)
{
    __shared__ __align__(16) uint8_t lds[(kBlock / kWave) * kInferLdsBytes];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    uint8_t *rows = lds + wave * kInferLdsBytes;
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < n;
    float L[16], x[16];
    float tot = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        L[m] = (valid && m < T.M) ? Lin[r * T.M + m] : 0.0f;
        x[m] = m < M.n_in ? __fmul_rn(L[m], M.in_scale[m]) : 0.0f;
        tot += L[m];
    }
    mlp_infer_wave(x, M, rows);
    if (!(valid && tot > 0.0f)) return;
    const int cell = cell_of(L, x, M);
    if (cell < 0) return;
    float ysum = 0.0f;
    for (int g = 0; g < T.G; ++g) ysum += Yin[(int64_t)g * n + r];
    float err = 0.0f;
    for (int g = 0; g < T.G; ++g) {
        float z = M.out_scale[g] * mlp_out(rows, lane, g);
#pragma unroll
        for (int m = 0; m < 16; ++m)
            if (m < T.M) z = fmaf(M.lin[g * T.M + m], L[m], z);
        const float pred = T.Wg[g] * expf(-z);
        const float ref = Yin[(int64_t)g * n + r];
        err = fmaxf(err, fabsf(pred - ref) / fmaxf(ref, kMlpShareFloor * ysum));
    }
    atomicMax(cell_err_bits + cell, __float_as_uint(err));   // non-negative floats order as their bits
    atomicAdd(cell_count + cell, 1);
}

// mbar[m] = sum_g W_g lin[g][m] / sum_g W_g, the spectrum-weighted mean
// attenuation of material m (zero beyond n_mat).
__global__ void k_mlp_mbar(SpecTables T, const float *__restrict__ lin, float *__restrict__ mbar)
{
    const int m = threadIdx.x;
    if (m >= FCAT_MLP_MAX_IO) return;
    double a = 0.0, b = 0.0;
    if (m < T.M)
        for (int g = 0; g < T.G; ++g) {
            a += (double)T.Wg[g] * (double)lin[g * T.M + m];
            b += (double)T.Wg[g];
        }
    mbar[m] = m < T.M ? (float)(a / b) : 0.0f;
}

// Set-up statistics of a training set, pass 1: a fixed grid of kStatBlocks
// blocks strides over the samples; block b writes partial[b][kStatStride]:
// max_s L[s][m], max_s sum_m mbar_m L[s][m], and per group the sums of
// omega r^2 and omega (target and weight as in k_mlp_grad).
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) v += __shfl_xor(v, sh);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) v = fmaxf(v, __shfl_xor(v, sh));
    return v;
}

__global__ __launch_bounds__(kBlock) void k_mlp_stats(SpecTables T, const float *__restrict__ lin,
                                                      const float *__restrict__ mbar, const float *__restrict__ Lin,
                                                      const float *__restrict__ Yin, int64_t n,
                                                      float *__restrict__ partial)
{
    __shared__ float red[kBlock / kWave][kStatStride];
    float mx[16], a[16], b[16], tmax = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) mx[k] = a[k] = b[k] = 0.0f;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (int64_t)kStatBlocks * kBlock) {
        float L[16], tau = 0.0f;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            L[m] = m < T.M ? Lin[s * T.M + m] : 0.0f;
            mx[m] = fmaxf(mx[m], L[m]);
            if (m < T.M) tau = fmaf(mbar[m], L[m], tau);
        }
        tmax = fmaxf(tmax, tau);
        float ysum = 0.0f;
        for (int g = 0; g < T.G; ++g) ysum += Yin[(int64_t)g * n + s];
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            if (g < T.G) {
                const float y = Yin[(int64_t)g * n + s];
                const float f = fminf(1.0f, y / (kMlpShareFloor * ysum));
                if (f > 0.0f) {
                    float r = -logf(y / T.Wg[g]);
#pragma unroll
                    for (int m = 0; m < 16; ++m)
                        if (m < T.M) r -= lin[g * T.M + m] * L[m];
                    a[g] = fmaf(f * f, r * r, a[g]);
                    b[g] += f * f;
                }
            }
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float vm = wave_max(mx[k]), va = wave_sum(a[k]), vb = wave_sum(b[k]);
        if (lane == 0) {
            red[wave][k] = vm;
            red[wave][17 + k] = va;
            red[wave][33 + k] = vb;
        }
    }
    const float vt = wave_max(tmax);
    if (lane == 0) red[wave][16] = vt;
    __syncthreads();
    if (threadIdx.x < 49) {
        const int k = threadIdx.x;
        float v = red[0][k];
        for (int w = 1; w < kBlock / kWave; ++w) v = (k <= 16) ? fmaxf(v, red[w][k]) : v + red[w][k];
        partial[(int64_t)blockIdx.x * kStatStride + k] = v;
    }
}

// Pass 2: reduce the block records in a fixed order (deterministic).
__global__ void k_mlp_stats_final(const float *__restrict__ partial, int M, int G, float *__restrict__ in_scale,
                                  float *__restrict__ out_scale, float *__restrict__ tau_max)
{
    const int k = threadIdx.x;
    if (k < M) {
        float v = 0.0f;
        for (int b = 0; b < kStatBlocks; ++b) v = fmaxf(v, partial[(int64_t)b * kStatStride + k]);
        in_scale[k] = 1.0f / fmaxf(v, 1e-6f);
    }
    if (k == 16) {
        float v = 0.0f;
        for (int b = 0; b < kStatBlocks; ++b) v = fmaxf(v, partial[(int64_t)b * kStatStride + 16]);
        tau_max[0] = v;
    }
    if (k >= 32 && k - 32 < G) {
        const int g = k - 32;
        double sa = 0.0, sb = 0.0;
        for (int b = 0; b < kStatBlocks; ++b) {
            sa += partial[(int64_t)b * kStatStride + 17 + g];
            sb += partial[(int64_t)b * kStatStride + 33 + g];
        }
        out_scale[g] = fmaxf(1e-3f, (float)sqrt(sa / fmax(sb, 1e-30)));
    }
}

__global__ void k_mlp_cells(const unsigned *__restrict__ err_bits, const int *__restrict__ count, int ncell,
                            float threshold, int min_count, float *__restrict__ cell_err, uint8_t *__restrict__ cell_ok)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const float e = __uint_as_float(err_bits[c]);
    if (cell_err) cell_err[c] = count[c] > 0 ? e : INFINITY;
    cell_ok[c] = (count[c] >= min_count && e <= threshold) ? 1 : 0;
}

}  // namespace

int mlp_param_count(int n_in, int n_out) { return param_offsets(n_in, n_out).P; }

hipError_t launch_mlp_prep(const float *params, int n_in, int n_out, uint4 *frag, hipStream_t stream, bool training)
{
    const int nf = training ? kMlpTrainFrags : kMlpFrags;
    hipLaunchKernelGGL(k_mlp_prep, dim3((nf * kWave + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, params,
                       n_in, n_out, frag, nf);
    return hipGetLastError();
}

hipError_t launch_mlp_linear(const float *mu, const SpecTables &t, float *lin, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_linear, dim3((t.G * t.M + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, mu, t, lin);
    return hipGetLastError();
}

hipError_t launch_mlp_mbar(const SpecTables &t, const float *lin, float *mbar, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_mbar, dim3(1), dim3(64), 0, stream, t, lin, mbar);
    return hipGetLastError();
}

hipError_t launch_mlp_stats(const SpecTables &t, const float *lin, const float *mbar, const float *L, const float *Y,
                            int64_t n, float *partial, float *in_scale, float *out_scale, float *tau_max,
                            hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_stats, dim3(kStatBlocks), dim3(kBlock), 0, stream, t, lin, mbar, L, Y, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_stats_final, dim3(1), dim3(64), 0, stream, partial, t.M, t.G, in_scale, out_scale,
                       tau_max);
    return hipGetLastError();
}

hipError_t launch_count_slots_sum(const int *slots, int *counts, hipStream_t stream)
{
    hipLaunchKernelGGL(k_count_slots_sum, dim3(1), dim3(kCountSlots), 0, stream, slots, counts);
    return hipGetLastError();
}

hipError_t launch_project_rows_mlp(const TraceGeom &g, const SpecTables &t, const MlpTables &m, const float *flood,
                                   const float *scatter, int a0, int n_ang, float *Y, float *out, int *slots,
                                   hipStream_t stream)
{
    const int64_t waves = (int64_t)n_ang * tiles_per_angle_host(g);
    const int nblk = padded_blocks(waves);
#define FCAT_FUSED(MPV)                                                                                          \
    hipLaunchKernelGGL(k_project_rows_mlp<MPV>, dim3(nblk), dim3(kBlock), 0, stream, g, t, m, flood, scatter, a0, \
                       n_ang, nblk, Y, out, slots)
    switch (t.mp) {
    case 8: FCAT_FUSED(8); break;
    case 10: FCAT_FUSED(10); break;
    case 12: FCAT_FUSED(12); break;
    case 16: FCAT_FUSED(16); break;
    default: return hipErrorInvalidValue;
    }
#undef FCAT_FUSED
    return hipGetLastError();
}

hipError_t launch_mlp_spectral(const SpecTables &t, const MlpTables &m, const SurrogateIO &io, hipStream_t stream)
{
    const unsigned nblk = (unsigned)((io.n + kBlock - 1) / kBlock);
    if (t.mp == 8)
        hipLaunchKernelGGL(k_mlp_spectral<8>, dim3(nblk), dim3(kBlock), 0, stream, t, m, io);
    else if (t.mp == 10)
        hipLaunchKernelGGL(k_mlp_spectral<10>, dim3(nblk), dim3(kBlock), 0, stream, t, m, io);
    else if (t.mp == 12)
        hipLaunchKernelGGL(k_mlp_spectral<12>, dim3(nblk), dim3(kBlock), 0, stream, t, m, io);
    else if (t.mp == 16)
        hipLaunchKernelGGL(k_mlp_spectral<16>, dim3(nblk), dim3(kBlock), 0, stream, t, m, io);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const SpecTables &t, const MlpTables &m, const float *L, const float *Y, int64_t n_all,
                           const int32_t *order, int64_t base, int count, float *partial, float *loss_partial,
                           hipStream_t stream)
{
    const unsigned nblk = (unsigned)((count + kWave - 1) / kWave);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(kGradWaves * kWave), 0, stream, t, m, L, Y, n_all, order, base,
                       count, partial, loss_partial);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce_adam(const float *partial, int nparts, int P, float *grad, float *params, float *m,
                                  float *v, int step, float lr, float beta1, float beta2, float eps,
                                  const float *loss_partial, float loss_scale, float *loss_out, hipStream_t stream,
                                  const int *cnt, const uint32_t *inv, uint4 *frag)
{
    static_assert(kReduceWaves == 4, "the four partial sums are added in a fixed order");
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((P + kWave - 1) / kWave), dim3(kBlock), 0, stream, partial, nparts, P,
                       grad, params, m, v, step, lr, beta1, beta2, eps, loss_partial, loss_scale, loss_out, cnt, inv,
                       reinterpret_cast<uint16_t *>(frag));
    return hipGetLastError();
}

hipError_t launch_mlp_frag_inverse(int n_in, int n_out, int *cnt, uint32_t *inv, hipStream_t stream)
{
    const int P = mlp_param_count(n_in, n_out);
    hipError_t e = launch_zero_ints(cnt, P, stream);
    if (e != hipSuccess) return e;
    const int n = kMlpTrainFrags * kWave * 8;
    hipLaunchKernelGGL(k_mlp_frag_inverse, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, n_in, n_out, cnt,
                       inv);
    return hipGetLastError();
}

hipError_t launch_mlp_validate(const SpecTables &t, const MlpTables &m, const float *L, const float *Y, int64_t n,
                               unsigned *err_bits, int *count, hipStream_t stream)
{
    const unsigned nblk = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_mlp_validate, dim3(nblk), dim3(kBlock), 0, stream, t, m, L, Y, n, err_bits, count);
    return hipGetLastError();
}

hipError_t launch_mlp_cells(const unsigned *err_bits, const int *count, int ncell, float threshold, int min_count,
                            float *cell_err, uint8_t *cell_ok, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_cells, dim3((ncell + 63) / 64), dim3(64), 0, stream, err_bits, count, ncell, threshold,
                       min_count, cell_err, cell_ok);
    return hipGetLastError();
}

}  // namespace fcat
