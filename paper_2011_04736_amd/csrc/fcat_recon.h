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

// Cosine-weighted, ramp-filtered rows of n_ang projections (proj and filt
// [n_ang][nv][nu], filt may not alias proj).
hipError_t launch_fdk_filter(const FdkGeom &g, const float *proj, int n_ang, float *filt, hipStream_t stream);

// (cos b, sin b) of angles a0 .. a0 + n - 1 into cs (2 n floats): from the
// device array angles, or 2 pi a / n_angles when angles is null.
hipError_t launch_fdk_angles(const double *angles, int n_angles, int a0, int n, float2 *cs, hipStream_t stream);

// volume (+)= (pi / n_angles) sum over the n angles of cs of D^2 / U^2 times
// the bilinear sample of filt at the voxel's detector position.
hipError_t launch_fdk_backproject(const FdkGeom &g, const FdkGrid &v, const float *filt, const float2 *cs, int n,
                                  float weight, int accumulate, float *volume, hipStream_t stream);

}  // namespace fcat
