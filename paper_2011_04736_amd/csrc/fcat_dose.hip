// Dose estimate (Sec. II.H, Eqs. 6-7): the mean over the rays of a set of
// projections of the energy a photon of each bin deposits,
//   S[e] = sum_i (1 - exp(-P_i(e))),   P_i(e) = sum_m mu[m][e] L_i,m,
// then D_0[e] = E_e (mu_en/mu)_e S[e] / (N_i M) and D_p = sum_e phi_e D_0[e].
//
// Per-material path lengths of a chunk of angles come from the walk kernel.
// k_dose_rays stages a tile of rays in LDS, keeps only the rays that meet the
// phantom (a ray with L = 0 adds exactly 0), and gives each lane one energy
// bin: the lane reads the tile's path lengths as LDS broadcasts and holds
// its mu column in registers, so no cross-lane reduction is needed.  (Where
// E is not a multiple of the workgroup some lanes idle; splitting each bin's
// rays in stripes over those lanes, so that lanes read different rows of the
// tile, measured 1.2x slower on the 200-bin contrast workload.)  Sums
// run in FP64 per lane, per workgroup in a fixed order, and over workgroups
// in a fixed order, so the result does not depend on scheduling.
#include "fcat_internal.h"

namespace fcat {
namespace {

constexpr int kDoseTile = 256;   // rays staged per tile (one per lane when loading)

// 1 - exp(-P) for an optical depth P >= 0, to a few ulp also where P is
// small: Cody and Waite's reduction (W. J. Cody, W. Waite, Software Manual
// for the Elementary Functions, 1980) P = n ln 2 + r with |r| <= ln 2 / 2 and
// ln 2 split in a 16-bit head (n times the head is exact for n < 2^8), then
// 1 - exp(-P) = (1 - 2^-n) - 2^-n expm1(-r), with expm1 on the reduced range
// by its Taylor series to degree 8 (truncation below 2e-8 relative).  Depths
// beyond 64 are taken as 64, where the result rounds to 1 already; a NaN
// stays NaN.  (It replaced the library expm1f: 31 instead of 36 vector
// instructions per ray and bin, the dose kernel 0.61 -> 0.54 ms.)
__device__ __forceinline__ float one_minus_exp_neg(float P)
{
    constexpr float kLog2e = 1.44269504088896341f;
    constexpr float kLn2Hi = 0.693145751953125f;        // ln 2 rounded to 16 significant bits
    constexpr float kLn2Lo = 1.428606765330187e-06f;    // ln 2 - kLn2Hi, rounded
    const float p = P > 64.0f ? 64.0f : P;
    const float n = rintf(p * kLog2e);                  // in [0, 93]
    float x = fmaf(n, kLn2Hi, -p);                      // -r
    x = fmaf(n, kLn2Lo, x);
    float q = fmaf(x, 1.0f / 40320.0f, 1.0f / 5040.0f);
    q = fmaf(x, q, 1.0f / 720.0f);
    q = fmaf(x, q, 1.0f / 120.0f);
    q = fmaf(x, q, 1.0f / 24.0f);
    q = fmaf(x, q, 1.0f / 6.0f);
    q = fmaf(x, q, 0.5f);
    q = fmaf(x, q, 1.0f);
    q *= x;                                             // expm1(-r)
    const float s = ldexpf(1.0f, (int)(-n));            // 2^-n, exact
    return fmaf(-s, q, 1.0f - s);
}

// Workgroup b takes the tiles b, b + gridDim, ... (gridDim = kDoseBlocks or fewer).
template <int MP>
__global__ void __launch_bounds__(kBlock) k_dose_rays(const float *__restrict__ L, int64_t n_rays, int M,
                                                      const float *__restrict__ muT, int E, int64_t n_tiles,
                                                      double *__restrict__ partial)
{
    __shared__ float Lt[kDoseTile][MP];
    __shared__ int n_hit;
    const int lane = (int)(threadIdx.x % kWave);
    // each lane owns energy bins e = threadIdx.x + k kBlock and their sums
    // in this workgroup's row of partial (read and written by that lane only)
    double *__restrict__ mine = partial + (int64_t)blockIdx.x * E;
    for (int e = (int)threadIdx.x; e < E; e += kBlock) mine[e] = 0.0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        if (threadIdx.x == 0) n_hit = 0;
        __syncthreads();
        // stage the rays of the tile that meet the phantom
        const int64_t r = tile * kDoseTile + threadIdx.x;
        float l[MP];
        bool hit = false;
        const float *__restrict__ row = L + min(r, n_rays - 1) * M;   // clamped: loads without branches
#pragma unroll
        for (int m = 0; m < MP; ++m) {
            const float v = row[min(m, M - 1)];
            l[m] = (r < n_rays && m < M) ? v : 0.0f;
            hit |= l[m] != 0.0f;
        }
        const uint64_t mask = __ballot(hit);
        int base = 0;
        if (lane == 0 && mask) base = atomicAdd(&n_hit, __popcll(mask));
        base = __shfl(base, 0);
        if (hit) {
            const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
#pragma unroll
            for (int m = 0; m < MP; ++m) Lt[slot][m] = l[m];
        }
        __syncthreads();
        const int nh = n_hit;
        for (int e = (int)threadIdx.x; nh > 0 && e < E; e += kBlock) {
            float mu[MP];
#pragma unroll
            for (int m = 0; m < MP; ++m) mu[m] = muT[e * MP + m];
            double s = 0.0;
#pragma unroll 4
            for (int j = 0; j < nh; ++j) {
                float P = 0.0f;
#pragma unroll
                for (int m = 0; m < MP; ++m) P = fmaf(mu[m], Lt[j][m], P);
                s += (double)one_minus_exp_neg(P);
            }
            mine[e] += s;
        }
        __syncthreads();
    }
}

// S[e] += sum over the nblk workgroup partials, in a fixed order; one
// workgroup per energy bin.
__global__ void __launch_bounds__(kBlock) k_dose_sum(const double *__restrict__ partial, int nblk, int E,
                                                     double *__restrict__ S)
{
    __shared__ double red[kBlock];
    const int e = blockIdx.x;
    double s = 0.0;
    for (int b = (int)threadIdx.x; b < nblk; b += kBlock) s += partial[(int64_t)b * E + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) S[e] += red[0];
}

// D0[e] = E_e r_e S[e] / (N M); Dp = sum_e phi_e D0[e] (bin order).
__global__ void k_dose_final(const double *__restrict__ S, const float *__restrict__ energy,
                             const float *__restrict__ ratio, const float *__restrict__ phi, int E, double inv_nm,
                             double *__restrict__ D0, double *__restrict__ Dp)
{
    if (threadIdx.x != 0) return;
    double dp = 0.0;
    for (int e = 0; e < E; ++e) {
        const double d = (double)energy[e] * (double)ratio[e] * S[e] * inv_nm;
        D0[e] = d;
        dp += (double)phi[e] * d;
    }
    if (Dp) *Dp = dp;
}

__global__ void k_zero_doubles(double *__restrict__ x, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

}  // namespace

int dose_blocks(int64_t n_rays)
{
    const int64_t tiles = (n_rays + kDoseTile - 1) / kDoseTile;
    return (int)(tiles < kDoseBlocks ? (tiles > 0 ? tiles : 1) : kDoseBlocks);
}

hipError_t launch_dose_rays(const float *L, int64_t n_rays, int M, const SpecTables &t, double *partial,
                            hipStream_t stream)
{
    const int64_t n_tiles = (n_rays + kDoseTile - 1) / kDoseTile;
    const int nblk = dose_blocks(n_rays);
    switch (t.mp) {
    case 8:
        hipLaunchKernelGGL(k_dose_rays<8>, dim3(nblk), dim3(kBlock), 0, stream, L, n_rays, M, t.muT, t.E, n_tiles,
                           partial);
        break;
    case 10:
        hipLaunchKernelGGL(k_dose_rays<10>, dim3(nblk), dim3(kBlock), 0, stream, L, n_rays, M, t.muT, t.E, n_tiles,
                           partial);
        break;
    case 12:
        hipLaunchKernelGGL(k_dose_rays<12>, dim3(nblk), dim3(kBlock), 0, stream, L, n_rays, M, t.muT, t.E, n_tiles,
                           partial);
        break;
    case 16:
        hipLaunchKernelGGL(k_dose_rays<16>, dim3(nblk), dim3(kBlock), 0, stream, L, n_rays, M, t.muT, t.E, n_tiles,
                           partial);
        break;
    default:
        hipLaunchKernelGGL(k_dose_rays<32>, dim3(nblk), dim3(kBlock), 0, stream, L, n_rays, M, t.muT, t.E, n_tiles,
                           partial);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_dose_sum(const double *partial, int nblk, int E, double *S, hipStream_t stream)
{
    hipLaunchKernelGGL(k_dose_sum, dim3(E), dim3(kBlock), 0, stream, partial, nblk, E, S);
    return hipGetLastError();
}

hipError_t launch_dose_final(const double *S, const float *energy, const float *ratio, const float *phi, int E,
                             double inv_nm, double *D0, double *Dp, hipStream_t stream)
{
    hipLaunchKernelGGL(k_dose_final, dim3(1), dim3(kWave), 0, stream, S, energy, ratio, phi, E, inv_nm, D0, Dp);
    return hipGetLastError();
}

hipError_t launch_zero_doubles(double *x, int n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_doubles, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, x, n);
    return hipGetLastError();
}

}  // namespace fcat
