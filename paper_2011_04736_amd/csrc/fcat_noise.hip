// Noise and projection stage (Sec. II.G, Eq. 5): Poisson counts on the group
// signals, the object-free flood through the optical spread, and the
// conversion of the detected profiles back to projections.
//
// Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// SC'11), keyed by the 64-bit seed; the draw of pixel p, group g and angle a
// runs on the counters (p, g, a, j), j = 0, 1, ..., each giving two (u, v)
// pairs of open uniforms (w + 1/2) 2^-32.  Poisson variates use inversion
// below a mean of 16 and Hormann's transformed rejection (PTRS, 1993) above,
// in FP64 with no fused multiply-adds, so that the integer a draw returns is
// fixed by the IEEE operations of the method and not by the compiler.
#include "fcat_internal.h"

namespace fcat {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;  // round multipliers
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;  // key increments
constexpr double kInversionLimit = 16.0;
constexpr int kMaxCdfTerms = 256;
constexpr int kMaxAttempts = 64;

// ln(k!) for k = 0..15, correctly rounded.
__constant__ double kLnFactorial[16] = {
    0.0, 0.0, 0.6931471805599453, 1.791759469228055, 3.1780538303479458, 4.787491742782046,
    6.579251212010101, 8.525161361065415, 10.60460290274525, 12.801827480081469, 15.104412573075516,
    17.502307845873887, 19.987214495661885, 22.552163853123425, 25.19122118273868, 27.89927138384089};

__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    }
    return c;
}

__device__ inline double open_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// The (u, v) pairs of one draw, in order.
struct UniformPairs {
    uint4 ctr;
    uint32_t k0, k1;
    uint4 w;
    bool second;   // the block's second pair is pending

    __device__ UniformPairs(uint32_t pixel, uint32_t group, uint32_t angle, uint32_t key0, uint32_t key1)
        : ctr(make_uint4(pixel, group, angle, 0u)), k0(key0), k1(key1), w(), second(false) {}

    __device__ void next(double &u, double &v)
    {
        if (second) {
            u = open_uniform(w.z);
            v = open_uniform(w.w);
            second = false;
            return;
        }
        w = philox4x32_10(ctr, k0, k1);
        ctr.w += 1u;
        u = open_uniform(w.x);
        v = open_uniform(w.y);
        second = true;
    }
};

// ln(k!) for an integer k >= 0: the table, else Stirling's series for
// ln Gamma(k + 1) to the x^-7 term (truncation below 1e-14 from k = 16).
__device__ inline double ln_factorial(double k)
{
#pragma clang fp contract(off)
    if (k < 16.0) return kLnFactorial[(int)k];
    const double x = k + 1.0;
    const double r = 1.0 / x;
    const double r2 = r * r;
    const double series = r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0 - r2 * (1.0 / 1680.0))));
    return (x - 0.5) * log(x) - x + 0.9189385332046728 + series;
}

// One Poisson(lam) variate (0 for lam <= 0 or NaN).
__device__ double poisson(double lam, UniformPairs &pairs)
{
#pragma clang fp contract(off)
    if (!(lam > 0.0)) return 0.0;
    double u, v;
    if (lam < kInversionLimit) {
        // smallest k with u <= F(k), the CDF summed term by term
        pairs.next(u, v);
        double p = exp(-lam);
        double F = p;
        int k = 0;
        while (u > F && k < kMaxCdfTerms) {
            ++k;
            p = p * lam / (double)k;
            F = F + p;
        }
        return (double)k;
    }
    const double b = 0.931 + 2.53 * sqrt(lam);
    const double a = -0.059 + 0.02483 * b;
    const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
    const double v_r = 0.9277 - 3.6224 / (b - 2.0);
    const double log_lam = log(lam);
    const double log_inv_alpha = log(inv_alpha);
    for (int attempt = 0; attempt < kMaxAttempts; ++attempt) {
        pairs.next(u, v);
        const double U = u - 0.5;
        const double us = 0.5 - fabs(U);
        const double k = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && v <= v_r) return k;
        if (k < 0.0 || (us < 0.013 && v > us)) continue;
        if (log(v) + log_inv_alpha - log(a / (us * us) + b) <= -lam + k * log_lam - ln_factorial(k)) return k;
    }
    return floor(lam + 0.5);
}

// ---------------------------------------------------------------------------
// Single-precision pass.  The FP64 draw above costs several FP64 logarithms
// and divisions per variate.  The kernel takes the same decisions from FP32
// estimates and hands a draw to the FP64 pass only where an estimate lies
// within a bound on its error of the decision boundary (an integer for the
// floor, the FP64 threshold for a comparison); elsewhere the two agree.  The
// bounds cover the FP32 roundings (a few ulp per operation, with a factor of
// 4 or more of margin) and the FP64 pass's own roundings.  Comparisons of the
// uniforms with constants are exact, in integers: u = (w + 1/2) 2^-32, so
// min(u, 1 - u) = (m + 1/2) 2^-32 with m = min(w, ~w).

// Least m with (m + 1/2) 2^-32 >= c, for a constant c of (0, 1/2).
constexpr uint32_t uniform_threshold(double c)
{
    const double x = c * 4294967296.0 - 0.5;   // exact: power-of-two scaling, then a multiple of the ulp
    const uint32_t f = (uint32_t)x;
    return (double)f < x ? f + 1u : f;
}
constexpr uint32_t kWide = uniform_threshold(0.07);     // us >= 0.07  <=>  m >= kWide
constexpr uint32_t kTail = uniform_threshold(0.013);    // us < 0.013  <=>  m < kTail

// ln n! - (n + 1/2) ln n + n - ln(2 pi) / 2 for n = 1..15 (Stirling remainder).
__constant__ float kStirlingRemainder[16] = {
    0.0f, 0.0810614675283432f, 0.041340697556734085f, 0.027677925303578377f, 0.020790671929717064f,
    0.016644692048430443f, 0.013876128941774368f, 0.01189670991152525f, 0.010411265306174755f,
    0.00925546232610941f, 0.008330563083291054f, 0.007573675364255905f, 0.006942840293049812f,
    0.00640899408608675f, 0.005951370112597942f, 0.005554733332246542f};

__device__ inline float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }   // 1 ulp

__device__ inline float stirling_remainder(float n)
{
    if (n < 16.0f) return kStirlingRemainder[(int)n];
    const float r = rcpf(n);
    const float r2 = r * r;
    return r * (1.0f / 12.0f - r2 * (1.0f / 360.0f - r2 * (1.0f / 1260.0f)));
}

// x ln(x / m) + m - x without cancellation near x = m (Loader 2000, "Fast and
// accurate computation of binomial probabilities"), with a bound on its
// FP32 error in err.
__device__ inline float deviance_term(float x, float m, float &err)
{
    const float d = x - m;      // exact near x = m (Sterbenz)
    const float s2 = x + m;
    if (fabsf(d) < 0.1f * s2) {
        const float v = d * rcpf(s2);
        const float v2 = v * v;
        float ej = 2.0f * x * v;
        float s = d * v;
        ej *= v2;
        s += ej * (1.0f / 3.0f);
        ej *= v2;
        s += ej * (1.0f / 5.0f);
        ej *= v2;
        s += ej * (1.0f / 7.0f);
        ej *= v2;
        s += ej * (1.0f / 9.0f);
        ej *= v2;
        s += ej * (1.0f / 11.0f);
        err = fabsf(s) * 0x1p-18f;
        return s;
    }
    const float t = x * __logf(x * rcpf(m));
    err = (fabsf(t) + s2) * 0x1p-18f;
    return t + m - x;
}

// Per-draw constants of the transformed rejection (FP32 estimates).
struct PtrsConst {
    float b, a, a2, log_inv_alpha, v_r, log_lam;
};

__device__ inline PtrsConst ptrs_const(float lam)
{
    PtrsConst P;
    P.b = 0.931f + 2.53f * __builtin_amdgcn_sqrtf(lam);   // 1 ulp
    P.a = -0.059f + 0.02483f * P.b;
    P.a2 = 2.0f * P.a;
    P.log_inv_alpha = __logf(1.1239f + 1.1328f * rcpf(P.b - 3.4f));
    P.v_r = 0.9277f - 3.6224f * rcpf(P.b - 2.0f);
    P.log_lam = __logf(lam);
    return P;
}

enum AttemptVerdict { kReject = 0, kAccept = 1, kExact = 2, kRatioTest = 3 };

// One attempt of the transformed rejection from the words (wu, wv) of its
// pair.  kReject: rejected for certain; kAccept: k is the variate; kExact:
// an estimate is too close to its boundary; kRatioTest: only the ratio test
// is left, and ratio_test is false.
__device__ inline int ptrs_attempt(const PtrsConst &P, float lam, uint32_t wu, uint32_t wv, bool ratio_test,
                                   double &k)
{
    const uint32_t m = min(wu, ~wu);
    const bool wide = m >= kWide;
    if (!wide && m < kTail && wv > m) return kReject;   // rejected whatever k is
    const float usf = ((float)m + 0.5f) * 0x1p-32f;
    const float Uf = ((float)(int32_t)(wu ^ 0x80000000u) + 0.5f) * 0x1p-32f;
    const float D = (P.a2 * rcpf(usf) + P.b) * Uf;
    const double X = ((double)D + (double)lam) + 0.43;
    k = floor(X);
    const double errX = fabs((double)D) * 0x1p-18 + (fabs(X) + fabs((double)D)) * 0x1p-50 + 0x1p-40;
    if (X - k <= errX || k + 1.0 - X <= errX) return kExact;
    const float vf = ((float)wv + 0.5f) * 0x1p-32f;
    if (wide) {
        if (vf <= P.v_r - 0x1p-19f) return kAccept;
        if (vf <= P.v_r + 0x1p-19f) return kExact;
    }
    if (k < 0.0) return kReject;
    if (!ratio_test) return kRatioTest;
    if (k >= 16777216.0) return kExact;   // k no longer exact in FP32
    // ln(v) + ln(1/alpha) - ln(a / us^2 + b) <= ln of the Poisson pmf at k
    const float lv = __logf(vf);
    const float lh = __logf(P.a * rcpf(usf * usf) + P.b);
    const float lhs = lv + P.log_inv_alpha - lh;
    const float kf = (float)k;
    float rhs = -lam, err_d = 0.0f;
    if (k > 0.0) rhs = -stirling_remainder(kf) - deviance_term(kf, lam, err_d) - 0.5f * __logf(6.2831853f * kf);
    // the FP64 pass's own rounding grows with the terms it cancels
    const float mag = lam + kf * (fabsf(P.log_lam) + __logf(kf + 1.0f) + 1.0f);
    const float eps = 0x1p-15f + err_d + 0x1p-18f * (fabsf(lv) + fabsf(lh) + fabsf(rhs) + 1.0f) + mag * 0x1p-46f;
    if (rhs - lhs >= eps) return kAccept;
    if (lhs - rhs > eps) return kReject;
    return kExact;
}

// Inversion for lam < 16 in FP32: the variate, or -1 where u lies too close
// to a CDF value.  Walks the terms of the CDF while u > F(k) for certain.
__device__ inline int inversion_single(float lam, uint32_t wu)
{
    const float uf = ((float)wu + 0.5f) * 0x1p-32f;
    float term = expf(-lam);
    float F = term;
    for (int k = 0; k < kMaxCdfTerms - 1; ++k) {
        const float tol = F * (8.0f + 8.0f * (float)k) * 0x1p-24f + 0x1p-24f;
        const float d = uf - F;
        if (d <= -tol) return k;   // u <= F(k) for certain, and u > F(j) held for every j < k
        if (d <= tol) return -1;
        term = term * lam * rcpf((float)(k + 1));
        F += term;
    }
    return -1;
}

constexpr int kPoissonPerLane = 8;                        // first-pass draws per lane
constexpr int kPoissonSpan = kBlock * kPoissonPerLane;    // pixels per workgroup (< 2^11)
constexpr int kQueuedAttempts = 32;                       // attempts a queued draw may take (< 2^5)

// Appends one LDS list entry per lane with push set, one atomic per
// wavefront; returns this lane's slot (or -1).  Called by whole wavefronts.
__device__ inline int wave_push(int *count, bool push)
{
    const uint64_t mask = __ballot(push);
    if (mask == 0) return -1;
    const int lane = (int)(threadIdx.x % kWave);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int start = 0;
    if (lane == leader) start = atomicAdd(count, __popcll(mask));
    start = __shfl(start, leader);
    return push ? start + __popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

// Y[pl][p] <- n / scale[g], n ~ Poisson(float(scale[g] Y)) for the planes
// pl = pl0 + blockIdx.x / nchunk (plane pl is angle pl / G, group pl % G of
// the call); a workgroup owns kPoissonSpan consecutive pixels of a plane.
// Rejection sampling gives lanes different amounts of work, and a wavefront
// pays for its slowest lane, so the work goes in rounds that keep lanes in
// step: the first takes one attempt of every draw; the draws it leaves open
// (rejected, or needing the ratio test: about a fifth) are queued in LDS,
// and each further round gives every queued draw one attempt, all 256
// lanes sharing the queue; the few draws left to the FP64 pass run last.
__global__ void __launch_bounds__(kBlock, 8) k_poisson(float *__restrict__ Y, int64_t plane, int G, unsigned nchunk,
                                                       unsigned pl0, const float *__restrict__ scale, uint32_t key0,
                                                       uint32_t key1, int angle_base)
{
    __shared__ uint16_t queue[2][kPoissonSpan];   // open draws: pixel offset | next attempt << 11
    __shared__ uint16_t exact[kPoissonSpan];      // draws left to the FP64 pass
    __shared__ int n_queue[2], n_exact;
    const unsigned bl = blockIdx.x / nchunk;
    const unsigned pl = pl0 + bl;
    const int g = (int)(pl % (unsigned)G);
    const uint32_t angle = (uint32_t)(angle_base + (int)(pl / (unsigned)G));
    const float c = scale[g];
    if (!(c > 0.0f)) return;                      // uniform over the workgroup
    const int64_t base = (int64_t)(blockIdx.x - bl * nchunk) * kPoissonSpan;
    float *__restrict__ Yp = Y + (int64_t)pl * plane + base;
    const int span = (int)min((int64_t)kPoissonSpan, plane - base);
    const float rc = 1.0f / c;                    // counts back to signal: n / c within 2 ulp
    if (threadIdx.x == 0) {
        n_queue[0] = 0;
        n_exact = 0;
    }
    __syncthreads();
    for (int e = 0; e < kPoissonPerLane; ++e) {
        const int i = e * kBlock + (int)threadIdx.x;
        bool to_exact = false, to_queue = false;
        int next = 0;
        if (i < span) {
            const float lam = c * Yp[i];
            if (!(lam > 0.0f)) {
                Yp[i] = 0.0f;
            } else {
                const uint4 w = philox4x32_10(make_uint4((uint32_t)(base + i), (uint32_t)g, angle, 0u), key0, key1);
                if (lam < (float)kInversionLimit) {
                    const int k = inversion_single(lam, w.x);
                    if (k >= 0) Yp[i] = (float)k * rc;
                    else to_exact = true;
                } else {
                    const PtrsConst P = ptrs_const(lam);
                    double k;
                    const int v = ptrs_attempt(P, lam, w.x, w.y, false, k);
                    if (v == kAccept) Yp[i] = (float)k * rc;
                    else if (v == kExact) to_exact = true;
                    else {
                        to_queue = true;
                        next = v == kReject ? 1 : 0;
                    }
                }
            }
        }
        const int se = wave_push(&n_exact, to_exact);
        if (to_exact) exact[se] = (uint16_t)i;
        const int sq = wave_push(&n_queue[0], to_queue);
        if (to_queue) queue[0][sq] = (uint16_t)(i | next << 11);
    }
    int cur = 0;
    while (true) {
        __syncthreads();
        const int nq = n_queue[cur];
        if (nq == 0) break;                       // uniform: read after the barrier
        if (threadIdx.x == 0) n_queue[cur ^ 1] = 0;
        __syncthreads();
        for (int j0 = 0; j0 < nq; j0 += kBlock) {
            const int j = j0 + (int)threadIdx.x;
            bool to_exact = false, to_queue = false;
            int i = 0, t = 0;
            if (j < nq) {
                i = queue[cur][j] & 0x7FF;
                t = queue[cur][j] >> 11;
                const float lam = c * Yp[i];
                const PtrsConst P = ptrs_const(lam);
                const uint4 w = philox4x32_10(make_uint4((uint32_t)(base + i), (uint32_t)g, angle, (uint32_t)(t >> 1)),
                                              key0, key1);
                double k;
                const int v = ptrs_attempt(P, lam, (t & 1) ? w.z : w.x, (t & 1) ? w.w : w.y, true, k);
                if (v == kAccept) Yp[i] = (float)k * rc;
                else if (v == kReject && t + 1 < kQueuedAttempts) to_queue = true;
                else to_exact = true;
            }
            const int se = wave_push(&n_exact, to_exact);
            if (to_exact) exact[se] = (uint16_t)i;
            const int sq = wave_push(&n_queue[cur ^ 1], to_queue);
            if (to_queue) queue[cur ^ 1][sq] = (uint16_t)(i | (t + 1) << 11);
        }
        cur ^= 1;
    }
    const int ne = n_exact;
    for (int j = (int)threadIdx.x; j < ne; j += kBlock) {
        const int i = exact[j];
        UniformPairs pairs((uint32_t)(base + i), (uint32_t)g, angle, key0, key1);
        Yp[i] = (float)poisson((double)(c * Yp[i]), pairs) * rc;
    }
}

// c_g = H Phi_g / (Phi W_g), FP64 sums in bin order, 0 for a group without
// fluence or response.  One lane per group.
struct GroupStarts {
    int s[FCAT_MAX_GROUPS + 1];
};

__global__ void k_count_scale(const float *__restrict__ phi, const float *__restrict__ eta, GroupStarts gs, int E,
                              int G, double H, float *__restrict__ scale)
{
#pragma clang fp contract(off)
    const int g = threadIdx.x;
    if (g >= G) return;
    double Phi = 0.0;
    for (int e = 0; e < E; ++e) Phi = Phi + (double)phi[e];
    double Pg = 0.0, Wg = 0.0;
    for (int e = gs.s[g]; e < gs.s[g + 1]; ++e) {
        Pg = Pg + (double)phi[e];
        Wg = Wg + (double)phi[e] * (double)eta[e];
    }
    scale[g] = (Pg != 0.0 && Wg != 0.0) ? (float)((H * Pg) / (Phi * Wg)) : 0.0f;
}

// Object-free, scatter-free group signals Yf[g][p] = W_g I0[p].
__global__ void k_flood_groups(const float *__restrict__ Wg, const float *__restrict__ i0, int64_t plane, int G,
                               float *__restrict__ Yf)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= plane) return;
    const float f = i0 ? i0[p] : 1.0f;
    for (int g = 0; g < G; ++g) Yf[(int64_t)g * plane + p] = Wg[g] * f;
}

// proj[a][p] = -ln(max(out[a][p], floor) / flood[p]); blockIdx.y = angle.
__global__ void __launch_bounds__(kBlock) k_log_projection(const float *__restrict__ out,
                                                           const float *__restrict__ flood, int64_t plane,
                                                           float floor_, float *__restrict__ proj)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= plane) return;
    const int64_t i = (int64_t)blockIdx.y * plane + p;
    proj[i] = -logf(fmaxf(out[i], floor_) / flood[p]);
}

__global__ void k_fill(float *__restrict__ x, int n, float v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}

}  // namespace

// A dispatch holds at most 2^32 - 1 work-items per grid dimension: large
// calls are split into launches of whole planes.
constexpr uint64_t kMaxLaunchBlocks = ((uint64_t)1 << 32) / kBlock - 1;

hipError_t launch_poisson(float *Y, int n_ang, int G, int64_t plane, const float *scale, uint64_t seed,
                          int angle_base, hipStream_t stream)
{
    if (n_ang <= 0 || G <= 0 || plane <= 0) return hipSuccess;
    const uint64_t nchunk = (uint64_t)((plane + kPoissonSpan - 1) / kPoissonSpan);
    const uint64_t planes = (uint64_t)n_ang * (uint64_t)G;
    const uint64_t per_launch = kMaxLaunchBlocks / nchunk;   // whole planes per launch
    if (per_launch == 0) return hipErrorInvalidValue;
    for (uint64_t pl0 = 0; pl0 < planes; pl0 += per_launch) {
        const uint64_t np = planes - pl0 < per_launch ? planes - pl0 : per_launch;
        hipLaunchKernelGGL(k_poisson, dim3((unsigned)(np * nchunk)), dim3(kBlock), 0, stream, Y, plane, G,
                           (unsigned)nchunk, (unsigned)pl0, scale, (uint32_t)seed, (uint32_t)(seed >> 32),
                           angle_base);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_count_scale(const float *phi, const float *eta, const int *gstart, int E, int G, double H,
                              float *scale, hipStream_t stream)
{
    GroupStarts gs{};
    for (int g = 0; g <= G; ++g) gs.s[g] = gstart[g];
    hipLaunchKernelGGL(k_count_scale, dim3(1), dim3(kWave), 0, stream, phi, eta, gs, E, G, H, scale);
    return hipGetLastError();
}

hipError_t launch_flood_groups(const float *Wg, const float *i0, int64_t plane, int G, float *Yf, hipStream_t stream)
{
    hipLaunchKernelGGL(k_flood_groups, dim3((unsigned)((plane + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, Wg,
                       i0, plane, G, Yf);
    return hipGetLastError();
}

hipError_t launch_log_projection(const float *out, const float *flood, int n_ang, int64_t plane, float floor_,
                                 float *proj, hipStream_t stream)
{
    if (n_ang <= 0 || plane <= 0) return hipSuccess;
    const uint64_t nblk = (uint64_t)((plane + kBlock - 1) / kBlock);
    if (nblk > kMaxLaunchBlocks) return hipErrorInvalidValue;
    constexpr int kMaxY = 65535;
    for (int a0 = 0; a0 < n_ang; a0 += kMaxY) {
        const int na = n_ang - a0 < kMaxY ? n_ang - a0 : kMaxY;
        hipLaunchKernelGGL(k_log_projection, dim3((unsigned)nblk, (unsigned)na), dim3(kBlock), 0, stream,
                           out + (int64_t)a0 * plane, flood, plane, floor_, proj + (int64_t)a0 * plane);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fill(float *x, int n, float v, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, x, n, v);
    return hipGetLastError();
}

}  // namespace fcat
