// Detector optics (Sec. II.B, Sec. IV.B): the spectrum-weighted effective
// PSF, the presampled MTF of a tilted slit, and Richardson-Lucy
// deconvolution (Richardson 1972; Lucy 1974) with the PSF.  The slit and LSF
// arithmetic runs in FP64 with no fused multiply-adds, so that the bin a
// pixel falls in is decided as the IEEE operations of the definition decide
// it; the images themselves are FP32.
#include "fcat_optics.h"

namespace fcat {
namespace {

struct Starts {
    int s[FCAT_MAX_GROUPS + 1];
};

__global__ void k_effective_psf(const float *__restrict__ phi, const float *__restrict__ eta, Starts gs, int G,
                                const float *__restrict__ kernels, int k, float *__restrict__ out)
{
    __shared__ double W[FCAT_MAX_GROUPS];
    __shared__ double Wsum;
    if ((int)threadIdx.x < G) {
        double w = 0.0;
        for (int e = gs.s[threadIdx.x]; e < gs.s[threadIdx.x + 1]; ++e) w += (double)phi[e] * (double)eta[e];
        W[threadIdx.x] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int g = 0; g < G; ++g) t += W[g];
        Wsum = t;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < k * k; i += kBlock) {
        double a = 0.0;
        for (int g = 0; g < G; ++g) a += W[g] * (double)kernels[(int64_t)g * k * k + i];
        out[i] = (float)(a / Wsum);
    }
}

// Area of the p x p square centred at 0 where a x + b y <= t (a, b != 0):
// a x + b y is the sum of two uniform variables of widths |a| p and |b| p,
// whose distribution function is a signed sum of four squared ramps.
__device__ inline double halfplane_area(double t, double a, double b, double p)
{
#pragma clang fp contract(off)
    const double A = fabs(a) * p, B = fabs(b) * p;
    const double s0 = -(A + B) / 2.0;
    const double u = t - s0;
    const double r0 = fmax(u, 0.0), r1 = fmax(u - A, 0.0), r2 = fmax(u - B, 0.0), r3 = fmax(u - A - B, 0.0);
    return (r0 * r0 - r1 * r1 - r2 * r2 + r3 * r3) / (2.0 * A * B) * p * p;
}

__device__ inline double pixel_distance(const SlitGeom &s, int i, int j)
{
#pragma clang fp contract(off)
    const double x = ((double)j - (double)(s.n_cols - 1) / 2.0) * s.pitch;
    const double y = ((double)i - (double)(s.n_rows - 1) / 2.0) * s.pitch;
    return s.cos_t * x + s.sin_t * y;
}

__global__ void k_slit_image(SlitGeom s, float *__restrict__ image)
{
#pragma clang fp contract(off)
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)s.n_rows * s.n_cols) return;
    const int i = (int)(idx / s.n_cols), j = (int)(idx % s.n_cols);
    const double d = pixel_distance(s, i, j);
    const double hi = halfplane_area(s.width / 2.0 - d, s.cos_t, s.sin_t, s.pitch);
    const double lo = halfplane_area(-s.width / 2.0 - d, s.cos_t, s.sin_t, s.pitch);
    image[idx] = (float)((hi - lo) / (s.pitch * s.pitch));
}

// One lane per bin: the mean of the pixels whose centre is nearest to the
// bin's distance, summed in pixel order (FP64).
__global__ void k_slit_lsf(SlitGeom s, const float *__restrict__ image, double *__restrict__ lsf,
                           int *__restrict__ count)
{
#pragma clang fp contract(off)
    const int bi = blockIdx.x * kBlock + (int)threadIdx.x;
    if (bi >= s.n_bins) return;
    const int64_t b = (int64_t)s.b_min + bi;
    double sum = 0.0;
    int n = 0;
    for (int i = 0; i < s.n_rows; ++i) {
        for (int j = 0; j < s.n_cols; ++j) {
            const double d = pixel_distance(s, i, j);
            if ((int64_t)floor(d / s.h + 0.5) == b) {
                sum += (double)image[(int64_t)i * s.n_cols + j];
                ++n;
            }
        }
    }
    lsf[bi] = n ? sum / (double)n : 0.0;
    count[bi] = n;
}

// One lane per frequency: |sum_b LSF_b e^{-2 pi i f d_b}| / |sum_b LSF_b| over
// the non-empty bins, in bin order.
__global__ void k_slit_mtf(SlitGeom s, const double *__restrict__ lsf, const int *__restrict__ count,
                           const double *__restrict__ freqs, int n_freq, double *__restrict__ mtf)
{
#pragma clang fp contract(off)
    const int fi = blockIdx.x * kBlock + (int)threadIdx.x;
    if (fi >= n_freq) return;
    const double f = freqs[fi];
    double re = 0.0, im = 0.0, tot = 0.0;
    for (int bi = 0; bi < s.n_bins; ++bi) {
        if (!count[bi]) continue;
        const double d = (double)(s.b_min + bi) * s.h;
        const double ph = -2.0 * 3.141592653589793 * f * d;
        re += lsf[bi] * cos(ph);
        im += lsf[bi] * sin(ph);
        tot += lsf[bi];
    }
    mtf[fi] = sqrt(re * re + im * im) / fabs(tot);
}

__global__ void k_flip_kernel(const float *__restrict__ kernel, int k, float *__restrict__ flipped)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < k * k) flipped[i] = kernel[k * k - 1 - i];
}

__global__ void k_fill_value(float *__restrict__ x, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) x[i] = v;
}

__global__ void k_rl_ratio(const float *__restrict__ d, float *__restrict__ c, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float ci = c[i];
        c[i] = ci > 0.0f ? d[i] / ci : 0.0f;
    }
}

__global__ void k_rl_update(float *__restrict__ u, const float *__restrict__ t, const float *__restrict__ norm,
                            int64_t plane, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        u[i] = u[i] * t[i] / norm[i % plane];
}

unsigned stream_blocks(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

hipError_t launch_effective_psf(const float *phi, const float *eta, const int *gstart, int G, const float *kernels,
                                int k, float *out, hipStream_t stream)
{
    Starts gs{};
    for (int g = 0; g <= G; ++g) gs.s[g] = gstart[g];
    hipLaunchKernelGGL(k_effective_psf, dim3(1), dim3(kBlock), 0, stream, phi, eta, gs, G, kernels, k, out);
    return hipGetLastError();
}

hipError_t launch_slit_image(const SlitGeom &s, float *image, hipStream_t stream)
{
    const int64_t n = (int64_t)s.n_rows * s.n_cols;
    hipLaunchKernelGGL(k_slit_image, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, s, image);
    return hipGetLastError();
}

hipError_t launch_slit_lsf(const SlitGeom &s, const float *image, double *lsf, int *count, hipStream_t stream)
{
    hipLaunchKernelGGL(k_slit_lsf, dim3((s.n_bins + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, s, image, lsf,
                       count);
    return hipGetLastError();
}

hipError_t launch_slit_mtf(const SlitGeom &s, const double *lsf, const int *count, const double *freqs, int n_freq,
                           double *mtf, hipStream_t stream)
{
    hipLaunchKernelGGL(k_slit_mtf, dim3((n_freq + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, s, lsf, count,
                       freqs, n_freq, mtf);
    return hipGetLastError();
}

hipError_t launch_flip_kernel(const float *kernel, int k, float *flipped, hipStream_t stream)
{
    hipLaunchKernelGGL(k_flip_kernel, dim3((k * k + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, kernel, k,
                       flipped);
    return hipGetLastError();
}

hipError_t launch_fill_value(float *x, int64_t n, float v, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fill_value, dim3(stream_blocks(n)), dim3(kBlock), 0, stream, x, n, v);
    return hipGetLastError();
}

hipError_t launch_rl_ratio(const float *d, float *c, int64_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_rl_ratio, dim3(stream_blocks(n)), dim3(kBlock), 0, stream, d, c, n);
    return hipGetLastError();
}

hipError_t launch_rl_update(float *u, const float *t, const float *norm, int64_t plane, int64_t n,
                            hipStream_t stream)
{
    hipLaunchKernelGGL(k_rl_update, dim3(stream_blocks(n)), dim3(kBlock), 0, stream, u, t, norm, plane, n);
    return hipGetLastError();
}

}  // namespace fcat
