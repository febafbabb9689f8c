// Internal declarations of the detector-optics stage (fcat_optics.hip):
// effective PSF, tilted-slit presampled MTF, Richardson-Lucy deconvolution.
// Not part of the public interface (include/fcat.h is).
#pragma once

#include "fcat_internal.h"

namespace fcat {

// K = sum_g W_g K_g / sum_g W_g with W_g = sum_{e in g} phi_e eta_e (FP64 sums).
hipError_t launch_effective_psf(const float *phi, const float *eta, const int *gstart, int G, const float *kernels,
                                int k, float *out, hipStream_t stream);

// Tilted slit: geometry shared by the image, the LSF bins and the MTF.
struct SlitGeom {
    double pitch, width, cos_t, sin_t, h;   // h = pitch / oversample
    int n_rows, n_cols, b_min, n_bins;
};

hipError_t launch_slit_image(const SlitGeom &s, float *image, hipStream_t stream);
hipError_t launch_slit_lsf(const SlitGeom &s, const float *image, double *lsf, int *count, hipStream_t stream);
hipError_t launch_slit_mtf(const SlitGeom &s, const double *lsf, const int *count, const double *freqs, int n_freq,
                           double *mtf, hipStream_t stream);

// Richardson-Lucy pieces: the flipped kernel, a fill, the ratio d / c (0
// where c <= 0, in place over c) and the update u <- u t / norm.
hipError_t launch_flip_kernel(const float *kernel, int k, float *flipped, hipStream_t stream);
hipError_t launch_fill_value(float *x, int64_t n, float v, hipStream_t stream);
hipError_t launch_rl_ratio(const float *d, float *c, int64_t n, hipStream_t stream);
hipError_t launch_rl_update(float *u, const float *t, const float *norm, int64_t plane, int64_t n,
                            hipStream_t stream);

}  // namespace fcat
