// Internal declarations of the FDK reconstruction (fcat_fdk.hip).  Not part
// of the public interface (include/fcat.h is).
#pragma once

#include "fcat_internal.h"

namespace fcat {

// Detector and scan description the FDK kernels need (host-built).
struct FdkGeom {
    float D;              // SID
    float scale;          // SDD / SID: virtual (axis) to real detector coordinates
    float du, dv, off_u, off_v, cu, cv;
    float tau;            // pixel pitch on the virtual detector, du SID / SDD
    float inv_du, inv_dv;
    int nu, nv;
};

// Voxel grid: centre of voxel (ix, iy, iz) at x0 + ix dx, ... .
struct FdkGrid {
    float x0, y0, z0, dx, dy, dz;
    int nx, ny, nz;
};

// Padded layout of filtered rows, used inside the whole reconstruction: per
// angle nv + 3 rows of fdk_padded_cols(nu) floats, detector row j at row
// j + 1; the rows of detector rows -1, nv, nv + 1 and the columns past nu
// hold zeros.
__host__ __device__ inline int fdk_padded_cols(int nu) { return nu < 2 ? 2 : nu; }
__host__ __device__ inline int64_t fdk_padded_plane(int nu, int nv) { return (int64_t)(nv + 3) * fdk_padded_cols(nu); }

// Ramp filter: outputs per lane, and the dynamic LDS one workgroup needs
// for rows of nu columns (the tap table, padded one word in eight, and the
// even/odd halves of the rows it filters).  Both the host check of nu and
// the launch use this one formula.
constexpr int kRampOut = 8;
constexpr size_t kFdkFilterMaxLds = 64 * 1024;
__host__ __device__ inline int fdk_filter_rows_per_block(int nu)
{
    const int nq = (nu + 1) / 2;
    const int ngrp = (nq + kRampOut - 1) / kRampOut;
    const int rpb = 256 / (2 * ngrp);
    return rpb < 1 ? 1 : rpb;
}
__host__ __device__ inline size_t fdk_filter_lds_bytes(int nu)
{
    const int nq = (nu + 1) / 2;
    const int ntab = 2 * nq + kRampOut + 1;
    return (size_t)(ntab + ntab / 8 + 1 + fdk_filter_rows_per_block(nu) * 2 * nq) * sizeof(float);
}

// Cosine-weighted, ramp-filtered rows of n_ang projections (proj
// [n_ang][nv][nu]; filt dense [n_ang][nv][nu] or, if padded, n_ang padded
// planes whose pads it leaves alone; filt may not alias proj).
hipError_t launch_fdk_filter(const FdkGeom &g, const float *proj, int n_ang, bool padded, float *filt,
                             hipStream_t stream);

// Zero the pads of n_ang padded planes.
hipError_t launch_fdk_pad(const FdkGeom &g, int n_ang, float *filt, hipStream_t stream);

// Quad layout of the padded rows, read by the back-projection: per angle
// nv + 2 rows of fdk_padded_cols(nu) - 1 float4, quad (j, c) = the padded
// values (j, c), (j, c + 1), (j + 1, c), (j + 1, c + 1): every bilinear
// sample is one aligned 16-byte load.
__host__ __device__ inline int64_t fdk_quad_plane(int nu, int nv)
{
    return (int64_t)(nv + 2) * (fdk_padded_cols(nu) - 1);
}

// quads (16-byte aligned) of n_ang padded planes (their pads zero).
hipError_t launch_fdk_quads(const FdkGeom &g, int n_ang, const float *filt, float4 *quads, hipStream_t stream);

// (cos b, sin b) of angles a0 .. a0 + n - 1 into cs (2 n floats): from the
// device array angles, or 2 pi a / n_angles when angles is null.
hipError_t launch_fdk_angles(const double *angles, int n_angles, int a0, int n, float2 *cs, hipStream_t stream);

// volume (+)= (pi / n_angles) sum over the n angles of cs of D^2 / U^2 times
// the bilinear sample of filt at the voxel's detector position.
// From dense filtered rows (filt) or, if filt is null, from quads.
hipError_t launch_fdk_backproject(const FdkGeom &g, const FdkGrid &v, const float *filt, const float4 *quads,
                                  const float2 *cs, int n, float weight, int accumulate, float *volume,
                                  hipStream_t stream);

}  // namespace fcat
