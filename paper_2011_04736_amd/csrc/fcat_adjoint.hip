// The projector of a real-valued voxel image and its transpose, for
// iterative reconstruction (Sec. II.F: a projection is the line integral
// along the source-to-pixel ray; Sec. II.G reconstructs from projections):
//   (A f)_r   = sum over the voxels k ray r crosses of l_rk f_k,
//   (A^T y)_k = sum over rays r of l_rk y_r,
// with l_rk the exact length of ray r in voxel k (Siddon's method).  Both
// walk every voxel of the ray with the same FP64 set-up and the same FP32
// plane stepping as the labelled projector (crossing k+1 of an axis at
// t0 + k dt, one rounding), so A^T is the transpose of A up to FP32
// rounding.  One lane follows one ray, a wavefront a compact tile of
// detector pixels.  A^T adds each ray's weighted lengths into the image with
// hardware floating-point atomics, so its sums are not in a fixed order.
#include "fcat_device.h"

namespace fcat {
namespace {

template <bool BACK>
__global__ __launch_bounds__(kBlock) void k_image_rays(TraceGeom G, const float *__restrict__ image_in,
                                                       float *image_out, const float *__restrict__ proj_in,
                                                       float *__restrict__ proj_out, int a0, int n_ang,
                                                       int nblk_pad)
{
    const int blk = xcd_block(nblk_pad);
    const int wave = uniform(threadIdx.x >> 6);
    const int gw = blk * (kBlock / kWave) + wave;
    if (gw >= n_ang * tiles_per_angle(G)) return;
    const PixelOf px = pixel_of(G, gw, threadIdx.x & (kWave - 1));
    if (!px.valid) return;
    const int64_t pix = ((int64_t)px.al * G.nv + px.iv) * G.nu + px.iu;
    float y = 0.0f;
    if (BACK) {
        y = proj_in[pix];
        if (y == 0.0f) return;
    }
    double st, ct;
    sincos(angle_of(G, a0 + px.al), &st, &ct);
    Ray r{};
    if (!setup_ray(G, ct, st, px.iv, px.iu, r)) {
        if (!BACK) proj_out[pix] = 0.0f;
        return;
    }
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    int i0 = r.i0[0], i1 = r.i0[1], i2 = r.i0[2];
    int loc = (i2 * ny + i1) * nx + i0;
    const int dl0 = r.sgn[0], dl1 = r.sgn[1] * nx, dl2 = r.sgn[2] * nx * ny;
    float t0 = r.t0[0], t1 = r.t0[1], t2 = r.t0[2];
    float k0 = 0.0f, k1 = 0.0f, k2 = 0.0f;
    float tprev = 0.0f, sum = 0.0f, comp = 0.0f;
    const int max_steps = nx + ny + nz + 3;
    for (int s = 0; s < max_steps; ++s) {
        const float tn = fminf(fminf(t0, t1), fminf(t2, r.t_end));
        const float seg = tn - tprev;
        if (BACK) {
            if (seg > 0.0f) unsafeAtomicAdd(image_out + loc, y * seg);
        } else {
            // compensated sum of f_k l_k along the ray
            const float v = fmaf(seg, image_in[loc], -comp);
            const float nsum = sum + v;
            comp = (nsum - sum) - v;
            sum = nsum;
        }
        if (!(tn < r.t_end)) break;
        // the nearest crossing's axis steps (x before y before z on ties);
        // a step out of the grid (rounding at its face) ends the ray
        const bool cx = (t0 == tn), cy = (t1 == tn);
        const bool ey = cy && !cx, ez = !cx && !cy;
        i0 += cx ? r.sgn[0] : 0;
        i1 += ey ? r.sgn[1] : 0;
        i2 += ez ? r.sgn[2] : 0;
        if ((unsigned)i0 >= (unsigned)nx || (unsigned)i1 >= (unsigned)ny || (unsigned)i2 >= (unsigned)nz) break;
        const int dyz = ey ? dl1 : dl2;
        loc += cx ? dl0 : dyz;
        k0 += cx ? 1.0f : 0.0f;
        k1 += ey ? 1.0f : 0.0f;
        k2 += ez ? 1.0f : 0.0f;
        t0 = fmaf(k0, r.dt[0], r.t0[0]);
        t1 = fmaf(k1, r.dt[1], r.t0[1]);
        t2 = fmaf(k2, r.dt[2], r.t0[2]);
        tprev = tn;
    }
    if (!BACK) proj_out[pix] = sum;
}

int image_blocks(const TraceGeom &g, int n_ang)
{
    const int64_t waves = (int64_t)n_ang * tiles_per_angle_host(g);
    const int64_t nblk = (waves + (kBlock / kWave) - 1) / (kBlock / kWave);
    return (int)((nblk + kXcds - 1) / kXcds * kXcds);
}

}  // namespace

hipError_t launch_image_project(const TraceGeom &g, const float *image, int a0, int n_ang, float *proj,
                                hipStream_t stream)
{
    const int nblk = image_blocks(g, n_ang);
    hipLaunchKernelGGL(k_image_rays<false>, dim3(nblk), dim3(kBlock), 0, stream, g, image, nullptr, nullptr, proj,
                       a0, n_ang, nblk);
    return hipGetLastError();
}

hipError_t launch_image_backproject(const TraceGeom &g, const float *proj, int a0, int n_ang, float *image,
                                    hipStream_t stream)
{
    const int nblk = image_blocks(g, n_ang);
    hipLaunchKernelGGL(k_image_rays<true>, dim3(nblk), dim3(kBlock), 0, stream, g, nullptr, image, proj, nullptr,
                       a0, n_ang, nblk);
    return hipGetLastError();
}

}  // namespace fcat
