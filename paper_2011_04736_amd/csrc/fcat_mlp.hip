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
// Every product runs on v_mfma_f32_16x16x32_bf16: weights, inputs and hidden
// activations are rounded to BF16 (nearest even), accumulation is FP32.  One
// wavefront handles 64 rays or samples; the activations pass between layers
// through LDS (the matrix-core output layout is the transpose of the input
// layout the next layer needs).  Training runs forward and backward on the
// same 64-sample tiles and writes one gradient partial per wavefront; the
// Adam kernel sums the partials in a fixed order, so training is
// deterministic.
#include "fcat_device.h"

namespace fcat {
namespace {

constexpr int H = FCAT_MLP_HIDDEN;     // 64
constexpr int SX = 40;                 // row stride (BF16) of 32-wide K buffers
constexpr int SH = 72;                 // row stride (BF16) of 64-wide K buffers
constexpr int SO = 17;                 // row stride (FP32) of the 16-wide output buffer

// B-operand fragment index (in units of 64 lanes) of each weight view.
constexpr int kFragW1 = 0;    // [ct 0..3][kb 0]      W1[n][k], k < n_in
constexpr int kFragW2 = 4;    // [ct 0..3][kb 0..1]   W2[n][k]
constexpr int kFragW3 = 12;   // [ct 0][kb 0..1]      W3[n][k], n < n_out
constexpr int kFragW3b = 14;  // [ct 0..3][kb 0]      B[o][h2] = W3[o][h2]   (dH2 = dZ3 W3)
constexpr int kFragW2b = 18;  // [ct 0..3][kb 0..1]   B[h2][h1] = W2[h2][h1] (dH1 = dZ2 W2)

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

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }

__device__ __forceinline__ float dsilu(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward pass of the 64 rays of the wavefront.  x (n_in values per lane)
// goes in; the n_out outputs of the ray of lane l come back in O[l][0..n_out).
__device__ __forceinline__ void mlp_infer_wave(const float (&x)[16], const MlpTables &M, uint16_t *X,
                                               uint16_t *Hb, float *O)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane >> 4, r16 = lane & 15;
    const Offsets off = param_offsets(M.n_in, M.n_out);
    const float *P = M.params;
#pragma unroll
    for (int k = 0; k < 32; k += 2) {
        const uint32_t lo = k < 16 ? bf16_rne(x[k]) : 0u;
        const uint32_t hi = k + 1 < 16 ? bf16_rne(x[k + 1]) : 0u;
        *reinterpret_cast<uint32_t *>(X + lane * SX + k) = lo | (hi << 16);
    }
    wave_sync_lds();
    // layer 1: [64 x 32] x [32 x 64]
    floatx4 acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const bf16x8 a = lds_frag(X, SX, 16 * rt + r16, 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW1 + ct, lane),
                                                                  floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const float b = P[off.b1 + 16 * ct + r16];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                Hb[(16 * rt + 4 * q + i) * SH + 16 * ct + r16] = (uint16_t)bf16_rne(silu(acc[rt][ct][i] + b));
    }
    wave_sync_lds();
    // layer 2: [64 x 64] x [64 x 64]
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 a = lds_frag(Hb, SH, 16 * rt + r16, 32 * kb + 8 * q);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, frag_of(M.frag, kFragW2 + ct * 2 + kb, lane), acc[rt][ct], 0, 0, 0);
        }
    wave_sync_lds();
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const float b = P[off.b2 + 16 * ct + r16];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                Hb[(16 * rt + 4 * q + i) * SH + 16 * ct + r16] = (uint16_t)bf16_rne(silu(acc[rt][ct][i] + b));
    }
    wave_sync_lds();
    // layer 3: [64 x 64] x [64 x 16]
    floatx4 o3[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        o3[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            o3[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_frag(Hb, SH, 16 * rt + r16, 32 * kb + 8 * q),
                                                             frag_of(M.frag, kFragW3 + kb, lane), o3[rt], 0, 0, 0);
    }
    const float b3 = r16 < M.n_out ? P[off.b3 + r16] : 0.0f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) O[(16 * rt + 4 * q + i) * SO + r16] = o3[rt][i] + b3;
    wave_sync_lds();
}

// Per-wavefront LDS of the forward pass; the output buffer reuses the input
// buffer, which is dead after the first layer.
struct InferLds {
    union {
        uint16_t X[kWave * SX];
        float O[kWave * SO];
    };
    uint16_t Hb[kWave * SH];
};

// ------------------------------------------------------------ kernels

// B-operand fragments of every weight view (FP32 master -> BF16).
__global__ __launch_bounds__(kBlock) void k_mlp_prep(const float *__restrict__ params, int n_in, int n_out,
                                                     uint4 *__restrict__ frag)
{
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= kMlpFrags * kWave) return;
    const int f = idx / kWave, lane = idx % kWave;
    const int q = lane >> 4, r16 = lane & 15;
    const Offsets off = param_offsets(n_in, n_out);
    uint32_t h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float v = 0.0f;
        if (f < kFragW2) {                       // W1[n][k]
            const int n = 16 * (f - kFragW1) + r16, k = 8 * q + j;
            if (k < n_in) v = params[off.W1 + n * n_in + k];
        } else if (f < kFragW3) {                // W2[n][k]
            const int ct = (f - kFragW2) / 2, kb = (f - kFragW2) % 2;
            const int n = 16 * ct + r16, k = 32 * kb + 8 * q + j;
            v = params[off.W2 + n * H + k];
        } else if (f < kFragW3b) {               // W3[n][k]
            const int kb = f - kFragW3;
            const int n = r16, k = 32 * kb + 8 * q + j;
            if (n < n_out) v = params[off.W3 + n * H + k];
        } else if (f < kFragW2b) {               // B[k = o][n = h2] = W3[o][h2]
            const int n = 16 * (f - kFragW3b) + r16, k = 8 * q + j;
            if (k < n_out) v = params[off.W3 + k * H + n];
        } else {                                 // B[k = h2][n = h1] = W2[h2][h1]
            const int ct = (f - kFragW2b) / 2, kb = (f - kFragW2b) % 2;
            const int n = 16 * ct + r16, k = 32 * kb + 8 * q + j;
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

// Validated-domain test of one ray (see fcat_surrogate_t).
__device__ __forceinline__ bool in_domain(const float (&L)[16], const float (&x)[16], float tot, const MlpTables &M)
{
    bool ok = tot > 0.0f;
    int dom = 0;
    float best = -1.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        if (m < M.n_in) {
            ok = ok && x[m] <= 1.0f;
            if (L[m] > best) {
                best = L[m];
                dom = m;
            }
        }
    }
    const float b = floorf((float)FCAT_MLP_CELLS * (log10f(tot) - M.cell_lo) / (M.cell_hi - M.cell_lo));
    ok = ok && b >= 0.0f && b < (float)FCAT_MLP_CELLS;
    if (!ok) return false;
    return M.cell_ok[dom * FCAT_MLP_CELLS + (int)b] != 0;
}

// Spectral stage with the surrogate: L [n][M] in, group signals out.
template <int MP>
__global__ __launch_bounds__(kBlock) void k_mlp_spectral(SpecTables T, MlpTables M, SurrogateIO io)
{
    __shared__ __align__(16) InferLds lds[kBlock / kWave];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < io.n;
    float L[16], x[16];
    float tot = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        L[m] = (valid && m < T.M) ? io.L[r * T.M + m] : 0.0f;
        x[m] = m < M.n_in ? L[m] * M.in_scale[m] : 0.0f;
        tot += L[m];
    }
    const bool hit = valid && tot > 0.0f;
    const bool use = hit && (io.force_mlp || in_domain(L, x, tot, M));
    if (__ballot(use) != 0) mlp_infer_wave(x, M, lds[wave].X, lds[wave].Hb, lds[wave].O);
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
            float z = M.out_scale[g] * lds[wave].O[lane * SO + g];
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

// Forward + backward of one 64-sample tile per workgroup (one wavefront).
// Samples order[base + i], i < count; the loss is the mean over `count`
// samples and n_out outputs of omega (s f - r)^2, with r the residual
// target, s = out_scale and omega = min(1, Y_g / (1e-6 sum_g Y_g))^2.  Writes
// the gradient partial of the tile to partial[blockIdx.x][P] and its loss
// sum to loss_partial[blockIdx.x].
__global__ __launch_bounds__(kWave) void k_mlp_grad(SpecTables T, MlpTables M, const float *__restrict__ Lin,
                                                    const float *__restrict__ Yin, int64_t n_all,
                                                    const int32_t *__restrict__ order, int64_t base, int count,
                                                    float *__restrict__ partial, float *__restrict__ loss_partial)
{
    __shared__ __align__(16) TrainLds S;
    const int lane = threadIdx.x;
    const int q = lane >> 4, r16 = lane & 15;
    const Offsets off = param_offsets(M.n_in, M.n_out);
    const float *P = M.params;
    const int n_in = M.n_in, n_out = M.n_out;
    const int local = blockIdx.x * kWave + lane;
    const bool valid = local < count;
    const int64_t s = valid ? (int64_t)(order ? order[base + local] : base + local) : 0;
    const float inv_n = 1.0f / ((float)count * (float)n_out);

    // inputs and residual targets r_g = -ln(Y_g / W_g) - sum_m lin[g][m] L_m
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
            t = -logf(y / T.Wg[g]);
#pragma unroll
            for (int m = 0; m < 16; ++m)
                if (m < n_in) t -= M.lin[g * n_in + m] * L[m];
            const float f = fminf(1.0f, y / (1e-6f * ysum));
            om = f * f;
        }
        S.Tg[lane * SO + g] = t;
        S.Wt[lane * SO + g] = om;
    }
#pragma unroll
    for (int k = 0; k < 32; k += 2) {
        const uint32_t lo = k < 16 ? bf16_rne(x[k]) : 0u;
        const uint32_t hi = k + 1 < 16 ? bf16_rne(x[k + 1]) : 0u;
        *reinterpret_cast<uint32_t *>(S.X + lane * SX + k) = lo | (hi << 16);
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) S.XT[m * SH + lane] = (uint16_t)bf16_rne(x[m]);
    wave_sync_lds();

    // ---- forward
    floatx4 Z1[4][4], Z2[4][4], acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const bf16x8 a = lds_frag(S.X, SX, 16 * rt + r16, 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            Z1[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW1 + ct, lane),
                                                                 floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const float b = P[off.b1 + 16 * ct + r16];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                Z1[rt][ct][i] += b;
                const uint16_t h = (uint16_t)bf16_rne(silu(Z1[rt][ct][i]));
                const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
                S.H1[row * SH + col] = h;
                S.H1T[col * SH + row] = h;
            }
    }
    wave_sync_lds();
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) Z2[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 a = lds_frag(S.H1, SH, 16 * rt + r16, 32 * kb + 8 * q);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                Z2[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, frag_of(M.frag, kFragW2 + ct * 2 + kb, lane), Z2[rt][ct], 0, 0, 0);
        }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const float b = P[off.b2 + 16 * ct + r16];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                Z2[rt][ct][i] += b;
                const uint16_t h = (uint16_t)bf16_rne(silu(Z2[rt][ct][i]));
                const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
                S.H2[row * SH + col] = h;
                S.H2T[col * SH + row] = h;
            }
    }
    wave_sync_lds();
    floatx4 o3[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        o3[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            o3[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_frag(S.H2, SH, 16 * rt + r16, 32 * kb + 8 * q),
                                                             frag_of(M.frag, kFragW3 + kb, lane), o3[rt], 0, 0, 0);
    }

    // ---- output error dZ3 = 2 omega (s f - r) s / (count n_out)
    const float b3 = r16 < n_out ? P[off.b3 + r16] : 0.0f;
    const float osc = r16 < n_out ? M.out_scale[r16] : 0.0f;
    float lsum = 0.0f, db3 = 0.0f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * rt + 4 * q + i;
            const bool live = r16 < n_out && (int)(blockIdx.x * kWave + row) < count;
            const float om = live ? S.Wt[row * SO + r16] : 0.0f;
            const float d = live ? osc * (o3[rt][i] + b3) - S.Tg[row * SO + r16] : 0.0f;
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
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const bf16x8 a = lds_frag(S.X, SX, 16 * rt + r16, 8 * q);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, frag_of(M.frag, kFragW3b + ct, lane),
                                                                  floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
    float db2[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float g = acc[rt][ct][i] * dsilu(Z2[rt][ct][i]);
                db2[ct] += g;
                const uint16_t gb = (uint16_t)bf16_rne(g);
                const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
                S.H1[row * SH + col] = gb;       // dZ2 [sample][h2]
                S.H2[col * SH + row] = gb;       // dZ2 transposed [h2][sample]
            }
    wave_sync_lds();

    // ---- dH1 = dZ2 W2 ; dZ1 = dH1 * silu'(Z1)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 a = lds_frag(S.H1, SH, 16 * rt + r16, 32 * kb + 8 * q);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, frag_of(M.frag, kFragW2b + ct * 2 + kb, lane), acc[rt][ct], 0, 0, 0);
        }
    float db1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float g = acc[rt][ct][i] * dsilu(Z1[rt][ct][i]);
                db1[ct] += g;
                const int row = 16 * rt + 4 * q + i, col = 16 * ct + r16;
                S.D1T[col * SH + row] = (uint16_t)bf16_rne(g);   // dZ1 transposed [h1][sample]
            }
    wave_sync_lds();

    float *out = partial + (int64_t)blockIdx.x * off.P;
    // ---- dW3[o][h2] = sum_s dZ3[s][o] H2[s][h2]
    {
        floatx4 w3[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) w3[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 a = lds_frag(S.D3T, SH, r16, 32 * kb + 8 * q);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                w3[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, lds_frag(S.H2T, SH, 16 * ct + r16, 32 * kb + 8 * q), w3[ct], 0, 0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = 4 * q + i;
                if (o < n_out) out[off.W3 + o * H + 16 * ct + r16] = w3[ct][i];
            }
    }
    // ---- dW2[h2][h1] = sum_s dZ2[s][h2] H1[s][h1]
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 a = lds_frag(S.H2, SH, 16 * rt + r16, 32 * kb + 8 * q);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, lds_frag(S.H1T, SH, 16 * ct + r16, 32 * kb + 8 * q), acc[rt][ct], 0, 0, 0);
        }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[off.W2 + (16 * rt + 4 * q + i) * H + 16 * ct + r16] = acc[rt][ct][i];
    // ---- dW1[h1][m] = sum_s dZ1[s][h1] X[s][m]
    {
        floatx4 w1[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            w1[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                w1[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_frag(S.D1T, SH, 16 * rt + r16, 32 * kb + 8 * q),
                                                                 lds_frag(S.XT, SH, r16, 32 * kb + 8 * q), w1[rt],
                                                                 0, 0, 0);
        }
        if (r16 < n_in) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) out[off.W1 + (16 * rt + 4 * q + i) * n_in + r16] = w1[rt][i];
        }
    }
    // ---- biases: column sums over the 64 samples (reduce the 4 lane quarters)
    db3 += __shfl_xor(db3, 16);
    db3 += __shfl_xor(db3, 32);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        db2[ct] += __shfl_xor(db2[ct], 16);
        db2[ct] += __shfl_xor(db2[ct], 32);
        db1[ct] += __shfl_xor(db1[ct], 16);
        db1[ct] += __shfl_xor(db1[ct], 32);
    }
    if (q == 0) {
        if (r16 < n_out) out[off.b3 + r16] = db3;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            out[off.b2 + 16 * ct + r16] = db2[ct];
            out[off.b1 + 16 * ct + r16] = db1[ct];
        }
    }
    // ---- loss sum of the tile
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) lsum += __shfl_xor(lsum, sh);
    if (lane == 0) loss_partial[blockIdx.x] = lsum;
}

// grad[p] = sum_w partial[w][p]; optionally the Adam update of params
// (Kingma & Ba 2015, Algorithm 1) with bias correction for step t; loss_out
// (if given) receives sum_w loss_partial[w] * loss_scale.
__global__ __launch_bounds__(kBlock) void k_mlp_reduce_adam(const float *__restrict__ partial, int nparts, int P,
                                                            float *__restrict__ grad, float *__restrict__ params,
                                                            float *__restrict__ m, float *__restrict__ v, int step,
                                                            float lr, float beta1, float beta2, float eps,
                                                            const float *__restrict__ loss_partial, float loss_scale,
                                                            float *__restrict__ loss_out)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p == 0 && loss_out) {
        float l = 0.0f;
        for (int w = 0; w < nparts; ++w) l += loss_partial[w];
        *loss_out = l * loss_scale;
    }
    if (p >= P) return;
    float g = 0.0f;
    for (int w = 0; w < nparts; ++w) g += partial[(int64_t)w * P + p];
    if (grad) grad[p] = g;
    if (params) {
        const float mt = beta1 * m[p] + (1.0f - beta1) * g;
        const float vt = beta2 * v[p] + (1.0f - beta2) * g * g;
        m[p] = mt;
        v[p] = vt;
        const float mhat = mt / (1.0f - powf(beta1, (float)step));
        const float vhat = vt / (1.0f - powf(beta2, (float)step));
        params[p] -= lr * mhat / (sqrtf(vhat) + eps);
    }
}

// Held-out validation: per ray, the largest relative error over groups of
// the predicted primary signal, with a floor of 1e-6 of the ray's total
// signal; its maximum and the sample count per cell.
__global__ __launch_bounds__(kBlock) void k_mlp_validate(SpecTables T, MlpTables M, const float *__restrict__ Lin,
                                                         const float *__restrict__ Yin, int64_t n,
                                                         unsigned *__restrict__ cell_err_bits,
                                                         int *__restrict__ cell_count)
{
    __shared__ __align__(16) InferLds lds[kBlock / kWave];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = r < n;
    float L[16], x[16];
    float tot = 0.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        L[m] = (valid && m < T.M) ? Lin[r * T.M + m] : 0.0f;
        x[m] = m < M.n_in ? L[m] * M.in_scale[m] : 0.0f;
        tot += L[m];
    }
    mlp_infer_wave(x, M, lds[wave].X, lds[wave].Hb, lds[wave].O);
    if (!(valid && tot > 0.0f)) return;
    bool inside = true;
    int dom = 0;
    float best = -1.0f;
#pragma unroll
    for (int m = 0; m < 16; ++m)
        if (m < M.n_in) {
            inside = inside && x[m] <= 1.0f;
            if (L[m] > best) {
                best = L[m];
                dom = m;
            }
        }
    const float b = floorf((float)FCAT_MLP_CELLS * (log10f(tot) - M.cell_lo) / (M.cell_hi - M.cell_lo));
    if (!inside || !(b >= 0.0f && b < (float)FCAT_MLP_CELLS)) return;
    float ysum = 0.0f;
    for (int g = 0; g < T.G; ++g) ysum += Yin[(int64_t)g * n + r];
    float err = 0.0f;
    for (int g = 0; g < T.G; ++g) {
        float z = M.out_scale[g] * lds[wave].O[lane * SO + g];
#pragma unroll
        for (int m = 0; m < 16; ++m)
            if (m < T.M) z = fmaf(M.lin[g * T.M + m], L[m], z);
        const float pred = T.Wg[g] * expf(-z);
        const float ref = Yin[(int64_t)g * n + r];
        err = fmaxf(err, fabsf(pred - ref) / fmaxf(ref, 1e-6f * ysum));
    }
    const int cell = dom * FCAT_MLP_CELLS + (int)b;
    atomicMax(cell_err_bits + cell, __float_as_uint(err));   // non-negative floats order as their bits
    atomicAdd(cell_count + cell, 1);
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

hipError_t launch_mlp_prep(const float *params, int n_in, int n_out, uint4 *frag, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_prep, dim3((kMlpFrags * kWave + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, params,
                       n_in, n_out, frag);
    return hipGetLastError();
}

hipError_t launch_mlp_linear(const float *mu, const SpecTables &t, float *lin, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_linear, dim3((t.G * t.M + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, mu, t, lin);
    return hipGetLastError();
}

hipError_t launch_mlp_spectral(const SpecTables &t, const MlpTables &m, const SurrogateIO &io, hipStream_t stream)
{
    const unsigned nblk = (unsigned)((io.n + kBlock - 1) / kBlock);
    if (t.mp == 8)
        hipLaunchKernelGGL(k_mlp_spectral<8>, dim3(nblk), dim3(kBlock), 0, stream, t, m, io);
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
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(kWave), 0, stream, t, m, L, Y, n_all, order, base, count, partial,
                       loss_partial);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce_adam(const float *partial, int nparts, int P, float *grad, float *params, float *m,
                                  float *v, int step, float lr, float beta1, float beta2, float eps,
                                  const float *loss_partial, float loss_scale, float *loss_out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((P + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, partial, nparts, P,
                       grad, params, m, v, step, lr, beta1, beta2, eps, loss_partial, loss_scale, loss_out);
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
