// FDK reconstruction (Sec. II.G; Feldkamp, Davis and Kress 1984) of the
// circular cone-beam scan: cosine weight and ramp filter along detector rows,
// then voxel-driven weighted back-projection with bilinear interpolation.
//
// The ramp is the band-limited (Ram-Lak) kernel in the spatial domain: tap 0
// is 1 / (4 tau), odd taps -1 / (n^2 pi^2 tau), even taps zero.  An output
// of one parity therefore only sees inputs of the other parity (besides tap
// 0), so each row is split into its even and odd samples and each half is
// a plain Toeplitz product with the odd taps.  A lane computes 8 consecutive
// outputs of one half with the kernel taps in a register window that slides
// by one per input: one LDS read of an input (shared by the lanes of a row)
// and one of a tap per 8 FMAs.
#include "fcat_recon.h"

namespace fcat {
namespace {


// Work of one lane: outputs i0 .. i0 + kRampOut - 1 of half s (0: even
// samples, 1: odd samples) of row r of the workgroup.
// Output row (a, iv) starts at filt + a plane_out + (iv + row_off) su.
__global__ void __launch_bounds__(kBlock) k_fdk_filter(FdkGeom g, const float *__restrict__ proj, int n_rows,
                                                       int rows_per_block, int64_t plane_out, int row_off, int su,
                                                       float *__restrict__ filt)
{
    extern __shared__ float lds[];
    const int nq = (g.nu + 1) / 2;                   // samples per half (the odd half zero-padded)
    const int ngrp = (nq + kRampOut - 1) / kRampOut;
    const int ntab = 2 * nq + kRampOut + 1;
    // tab[j + j / 8] = G[j - nq], G[d] = h((2d - 1) tau) tau: one pad word per 8
    // makes the lanes' reads (8 entries apart) fall in different banks
    float *__restrict__ tab = lds;
    float *__restrict__ half = lds + ntab + ntab / 8 + 1;   // [rows_per_block][2][nq]
    const float pi2tau = 9.869604401089358f * g.tau;
    for (int j = (int)threadIdx.x; j < ntab; j += kBlock) {
        const float m = (float)(2 * (j - nq) - 1);   // odd offset
        tab[j + (j >> 3)] = -1.0f / (m * m * pi2tau);
    }
    const int row0 = blockIdx.x * rows_per_block;
    const int nr = min(rows_per_block, n_rows - row0);
    for (int k = (int)threadIdx.x; k < nr * 2 * nq; k += kBlock) {
        const int r = k / (2 * nq);
        const int rem = k - r * 2 * nq;
        const int s = rem / nq, l = rem - s * nq;
        const int iu = 2 * l + s;
        const int row = row0 + r;
        const int iv = row % g.nv;
        float v = 0.0f;
        if (iu < g.nu) {
            const float a = ((float)iu - g.cu) * g.du + g.off_u;
            const float c = ((float)iv - g.cv) * g.dv + g.off_v;
            const float av = a / g.scale, cvv = c / g.scale;
            v = proj[(int64_t)row * g.nu + iu] * (g.D * rsqrtf(g.D * g.D + av * av + cvv * cvv));
        }
        half[(r * 2 + s) * nq + l] = v;
    }
    __syncthreads();
    const float h0 = 0.25f / g.tau;
    for (int w = (int)threadIdx.x; w < nr * 2 * ngrp; w += kBlock) {
        const int r = w / (2 * ngrp);
        const int s = (w / ngrp) & 1;
        const int i0 = (w % ngrp) * kRampOut;
        const float *__restrict__ other = half + (r * 2 + (1 - s)) * nq;
        const float *__restrict__ self = half + (r * 2 + s) * nq;
        // out half s at i = h0 x_s[i] + sum_l G[i - l + s] x_(1-s)[l]
        const int base = i0 + s + nq;                // tab index of G[i0 + s - l] at l = 0
        float win[kRampOut], acc[kRampOut];
#pragma unroll
        for (int q = 0; q < kRampOut; ++q) {
            win[q] = tab[base + q + ((base + q) >> 3)];
            acc[q] = 0.0f;
        }
        // After input l the window takes G at j = base - 1 - l, stored at
        // j + j / 8.  With base - 1 = 8 hb + rho, input l = 8 t + u reads
        // 9 (hb - t) + rho - u - (u > rho): per block of 8 inputs a base
        // that steps by 9, and per input one subtraction of a lane constant.
        const int hb = (base - 1) >> 3, rho = (base - 1) & 7;
        int dlt[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) dlt[u] = u + (u > rho ? 1 : 0);
        int l = 0;
        for (int pb = 9 * hb + rho; l + 8 <= nq; l += 8, pb -= 9) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float xv = other[l + u];
#pragma unroll
                for (int q = 0; q < kRampOut; ++q) acc[q] = fmaf(win[q], xv, acc[q]);
#pragma unroll
                for (int q = kRampOut - 1; q > 0; --q) win[q] = win[q - 1];
                win[0] = tab[pb - dlt[u]];
            }
        }
        for (; l < nq; ++l) {
            const float xv = other[l];
#pragma unroll
            for (int q = 0; q < kRampOut; ++q) acc[q] = fmaf(win[q], xv, acc[q]);
#pragma unroll
            for (int q = kRampOut - 1; q > 0; --q) win[q] = win[q - 1];
            const int j = base - l - 1;
            win[0] = tab[j + (j >> 3)];
        }
        const int row = row0 + r;
        float *__restrict__ orow = filt + (int64_t)(row / g.nv) * plane_out + (int64_t)(row % g.nv + row_off) * su;
#pragma unroll
        for (int q = 0; q < kRampOut; ++q) {
            const int i = i0 + q;
            const int iu = 2 * i + s;
            if (i < nq && iu < g.nu) orow[iu] = fmaf(h0, self[i], acc[q]);
        }
    }
}

__global__ void k_fdk_angles(const double *__restrict__ angles, int n_angles, int a0, int n, float2 *__restrict__ cs)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double b = angles ? angles[a0 + i] : 6.283185307179586 * (double)(a0 + i) / (double)n_angles;
    double sb, cb;
    sincos(b, &sb, &cb);
    cs[i] = make_float2((float)cb, (float)sb);
}

constexpr int kBpZ = 16;       // slices a lane accumulates per pass
constexpr int kBpTileX = 64;   // workgroup tile: 64 x 4 columns (x fastest, one wavefront per row)

// Voxel-driven back-projection of filtered rows in the dense layout
// [n][nv][nu] (the caller's own rows): a lane owns one (x, y) column and zc <= kBpZ
// slices starting at blockIdx.z zc (the slices split evenly over gridDim.z),
// and loops over the angles.  The taps are read from global memory: the
// window of the detector a workgroup touches per angle is small and stays in
// the caches (staging it in LDS, one angle ahead with a barrier per angle,
// measured twice as slow on the 10-slice contrast grid).
__global__ void __launch_bounds__(kBlock) k_fdk_backproject_dense(FdkGeom g, FdkGrid v,
                                                                  const float *__restrict__ filt,
                                                                  const float2 *__restrict__ cs, int n, int zc,
                                                                  float weight, int accumulate,
                                                                  float *__restrict__ volume)
{
    const int ix = blockIdx.x * kBpTileX + (int)(threadIdx.x % kBpTileX);
    const int iy = blockIdx.y * (kBlock / kBpTileX) + (int)(threadIdx.x / kBpTileX);
    const int iz0 = blockIdx.z * zc;
    const int nzl = min(zc, v.nz - iz0);         // slices of this workgroup
    if (ix >= v.nx || iy >= v.ny) return;
    const float x = v.x0 + (float)ix * v.dx;
    const float y = v.y0 + (float)iy * v.dy;
    float acc[kBpZ];
#pragma unroll
    for (int q = 0; q < kBpZ; ++q) acc[q] = 0.0f;
    const int64_t plane = (int64_t)g.nu * g.nv;
    for (int a = 0; a < n; ++a) {
        const float2 c = cs[a];
        const float s = x * c.x + y * c.y;
        const float t = y * c.x - x * c.y;
        const float mag = g.D * __builtin_amdgcn_rcpf(g.D - s);   // D / U (1 ulp reciprocal)
        const float w = mag * mag;                                  // D^2 / U^2
        const float uf = (t * mag * g.scale - g.off_u) * g.inv_du + g.cu;
        const float fu0 = floorf(uf);
        const float fu = uf - fu0;
        const int i0 = (int)fu0;
        const bool cin0 = i0 >= 0 && i0 < g.nu, cin1 = i0 + 1 >= 0 && i0 + 1 < g.nu;
        const int c0 = min(max(i0, 0), g.nu - 1), c1 = min(max(i0 + 1, 0), g.nu - 1);
        const float *__restrict__ p = filt + (int64_t)a * plane;
        // detector row j interpolated along u at this column (taps outside
        // the detector count as 0); rows are clamped for the loads only
        auto row_value = [&](int j) {
            const int r = min(max(j, 0), g.nv - 1);
            const float a0 = cin0 ? p[r * g.nu + c0] : 0.0f;
            const float a1 = cin1 ? p[r * g.nu + c1] : 0.0f;
            const float val = fmaf(fu, a1 - a0, a0);
            return (j >= 0 && j < g.nv) ? val : 0.0f;
        };
        const float zstep = v.dz * mag * g.scale * g.inv_dv;   // detector rows per slice
        const float vf0 = ((v.z0 + (float)iz0 * v.dz) * mag * g.scale - g.off_v) * g.inv_dv + g.cv;
        // The slices of a column meet the detector at increasing rows, often
        // less than a row apart: the u-interpolated values of the current
        // row pair stay in registers, and a step of one row reuses the lower
        // one as the upper, so only the new row is read and interpolated.
        int rt = -(1 << 30);                    // row of the upper value held
        float top = 0.0f, bot = 0.0f;
#pragma unroll
        for (int q = 0; q < kBpZ; ++q) {
            if (q >= nzl) continue;             // uniform: the workgroup's slice count
            const float vf = vf0 + (float)q * zstep;
            const float fv0 = floorf(vf);
            const float fv = vf - fv0;
            const int j0 = (int)fv0;
            if (j0 != rt) {
                if (j0 == rt + 1)
                    top = bot;
                else
                    top = row_value(j0);
                bot = row_value(j0 + 1);
                rt = j0;
            }
            acc[q] = fmaf(w, fmaf(fv, bot - top, top), acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < kBpZ; ++q) {
        const int iz = iz0 + q;
        if (q < nzl) {
            float *o = volume + ((int64_t)iz * v.ny + iy) * v.nx + ix;
            *o = (accumulate ? *o : 0.0f) + weight * acc[q];
        }
    }
}


// Zero the pad rows (detector rows -1, nv, nv + 1) and pad columns (nu ..
// su - 1) of n planes in the padded layout.
__global__ void k_fdk_pad(float *__restrict__ filt, int n, int nu, int nv, int su)
{
    const int64_t per = 3 * (int64_t)su + (int64_t)nv * (su - nu);   // pad words per plane
    const int64_t plane = (int64_t)(nv + 3) * su;
    const int64_t total = per * n;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < total; k += (int64_t)gridDim.x * kBlock) {
        const int64_t a = k / per;
        int64_t r = k - a * per;
        int64_t idx;
        if (r < 3 * (int64_t)su) {
            const int which = (int)(r / su);                 // 0: row -1, 1: row nv, 2: row nv + 1
            const int c = (int)(r - (int64_t)which * su);
            idx = (int64_t)(which == 0 ? 0 : nv + which) * su + c;
        } else {
            r -= 3 * (int64_t)su;                            // only when su > nu
            const int w = su - nu;
            const int j = (int)(r / w);
            idx = (int64_t)(j + 1) * su + nu + (int)(r - (int64_t)j * w);
        }
        filt[a * plane + idx] = 0.0f;
    }
}

// Quads of the padded rows: lane per (plane, row j in [0, nv + 1], column c in
// [0, su - 2]), reading the padded plane coalesced and writing one float4.
__global__ void k_fdk_quads(const float *__restrict__ filt, int n, int nv, int su, float4 *__restrict__ quads)
{
    const int qc = su - 1;
    const int64_t per = (int64_t)(nv + 2) * qc;
    const int64_t plane = (int64_t)(nv + 3) * su;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < per * n; k += (int64_t)gridDim.x * kBlock) {
        const int64_t a = k / per;
        const int64_t r = k - a * per;
        const int j = (int)(r / qc), c = (int)(r - (int64_t)j * qc);
        const float *__restrict__ f = filt + a * plane + (int64_t)j * su + c;
        quads[k] = make_float4(f[0], f[1], f[su], f[su + 1]);
    }
}

// The back-projection of the whole reconstruction, from quads of the padded
// filtered rows.  A lane owns one (x, y) column and Z slices (Z = zc, the
// workgroup's share of the z extent; the last z block may own fewer, nzl:
// its extra slices read in-bounds quads and are not stored), with no branch
// and no bounds test per slice:
//  * the two columns of a sample are c0 and c0 + 1 with c0 clamped to
//    [0, su - 2]; their weights are the bilinear tent weights
//    max(0, 1 - |u - c|), so a tap off the detector gets weight 0 (or reads
//    a zero pad column);
//  * the row coordinate, counted in padded rows (detector row + 1), is
//    clamped to [0, nv + 1] (a NaN gives offset 0): a sample off the
//    detector then reads the zero pad rows, the value of a tap outside it.
// Per slice: the row and its fraction, one 24-bit address, one aligned
// 16-byte load and seven FMAs/adds; the per-angle terms are shared by the
// column's slices.  (On the 10-slice contrast grid the same branch-free loop
// reading the two rows as two 8-byte loads at 4-byte alignment measured
// 1.2x slower than the dense kernel, bound by its vector memory requests,
// and the dense kernel's reuse of rows between slices on the padded rows
// only 2% faster, held up by its load-to-use waits inside the branches.)
template <int Z>
__global__ void __launch_bounds__(kBlock) k_fdk_backproject(FdkGeom g, FdkGrid v, const float4 *__restrict__ quads,
                                                            const float2 *__restrict__ cs, int n, float weight,
                                                            int accumulate, float *__restrict__ volume)
{
    const int ix = blockIdx.x * kBpTileX + (int)(threadIdx.x % kBpTileX);
    const int iy = blockIdx.y * (kBlock / kBpTileX) + (int)(threadIdx.x / kBpTileX);
    const int iz0 = blockIdx.z * Z;
    const int nzl = min(Z, v.nz - iz0);          // slices of this workgroup that exist
    if (ix >= v.nx || iy >= v.ny) return;
    const float x = v.x0 + (float)ix * v.dx;
    const float y = v.y0 + (float)iy * v.dy;
    float acc[Z];
#pragma unroll
    for (int q = 0; q < Z; ++q) acc[q] = 0.0f;
    const int su = fdk_padded_cols(g.nu);
    const int64_t plane = fdk_quad_plane(g.nu, g.nv);
    const uint32_t row_bytes = (uint32_t)(su - 1) * sizeof(float4);   // < 2^24
    const float vmax = (float)(g.nv + 1);
    for (int a = 0; a < n; ++a) {
        const float2 c = cs[a];
        const float s = x * c.x + y * c.y;
        const float t = y * c.x - x * c.y;
        const float mag = g.D * __builtin_amdgcn_rcpf(g.D - s);   // D / U (1 ulp reciprocal)
        const float w = mag * mag;                                  // D^2 / U^2
        const float uf = (t * mag * g.scale - g.off_u) * g.inv_du + g.cu;
        const int c0 = min(max((int)floorf(uf), 0), su - 2);
        const float d = uf - (float)c0;
        const float w0 = fmaxf(1.0f - fabsf(d), 0.0f);
        const float w1 = fmaxf(1.0f - fabsf(d - 1.0f), 0.0f);
        const char *__restrict__ pa = reinterpret_cast<const char *>(quads + (int64_t)a * plane);
        const uint32_t cb = (uint32_t)c0 * sizeof(float4);
        const float zstep = v.dz * mag * g.scale * g.inv_dv;   // detector rows per slice
        // padded row coordinate (detector row + 1) of the first slice
        const float vf0 = ((v.z0 + (float)iz0 * v.dz) * mag * g.scale - g.off_v) * g.inv_dv + (g.cv + 1.0f);
#pragma unroll
        for (int q = 0; q < Z; ++q) {
            const float vf = __builtin_amdgcn_fmed3f(vf0 + (float)q * zstep, 0.0f, vmax);
            const float fl = floorf(vf);
            const float fv = vf - fl;
            // quad (row fl, column c0), fl in [0, nv + 1] (0 for a NaN)
            const float4 p = *reinterpret_cast<const float4 *>(
                pa + ((uint32_t)__umul24((uint32_t)(int)fl, row_bytes) + cb));
            const float top = fmaf(w1, p.y, w0 * p.x);
            const float bot = fmaf(w1, p.w, w0 * p.z);
            acc[q] = fmaf(w, fmaf(fv, bot - top, top), acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < Z; ++q) {
        const int iz = iz0 + q;
        if (q < nzl) {
            float *o = volume + ((int64_t)iz * v.ny + iy) * v.nx + ix;
            *o = (accumulate ? *o : 0.0f) + weight * acc[q];
        }
    }
}

}  // namespace

hipError_t launch_fdk_filter(const FdkGeom &g, const float *proj, int n_ang, bool padded, float *filt,
                             hipStream_t stream)
{
    const int su = padded ? fdk_padded_cols(g.nu) : g.nu;
    const int64_t plane_out = padded ? fdk_padded_plane(g.nu, g.nv) : (int64_t)g.nu * g.nv;
    const int rows = n_ang * g.nv;
    const int rpb = fdk_filter_rows_per_block(g.nu);
    const size_t lds = fdk_filter_lds_bytes(g.nu);
    if (lds > kFdkFilterMaxLds) return hipErrorInvalidValue;
    const int nblk = (rows + rpb - 1) / rpb;
    hipLaunchKernelGGL(k_fdk_filter, dim3(nblk), dim3(kBlock), lds, stream, g, proj, rows, rpb, plane_out,
                       padded ? 1 : 0, su, filt);
    return hipGetLastError();
}

hipError_t launch_fdk_angles(const double *angles, int n_angles, int a0, int n, float2 *cs, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fdk_angles, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, angles, n_angles, a0, n,
                       cs);
    return hipGetLastError();
}

hipError_t launch_fdk_pad(const FdkGeom &g, int n_ang, float *filt, hipStream_t stream)
{
    const int su = fdk_padded_cols(g.nu);
    const int64_t total = (3 * (int64_t)su + (int64_t)g.nv * (su - g.nu)) * n_ang;
    if (total == 0) return hipSuccess;
    const int64_t nblk = std::min<int64_t>((total + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_fdk_pad, dim3((unsigned)nblk), dim3(kBlock), 0, stream, filt, n_ang, g.nu, g.nv, su);
    return hipGetLastError();
}

hipError_t launch_fdk_quads(const FdkGeom &g, int n_ang, const float *filt, float4 *quads, hipStream_t stream)
{
    const int su = fdk_padded_cols(g.nu);
    const int64_t total = fdk_quad_plane(g.nu, g.nv) * n_ang;
    if (total == 0) return hipSuccess;
    const int64_t nblk = std::min<int64_t>((total + kBlock - 1) / kBlock, 16384);
    hipLaunchKernelGGL(k_fdk_quads, dim3((unsigned)nblk), dim3(kBlock), 0, stream, filt, n_ang, g.nv, su, quads);
    return hipGetLastError();
}

hipError_t launch_fdk_backproject(const FdkGeom &g, const FdkGrid &v, const float *filt, const float4 *quads,
                                  const float2 *cs, int n, float weight, int accumulate, float *volume,
                                  hipStream_t stream)
{
    const int nzb = (v.nz + kBpZ - 1) / kBpZ;        // passes over z
    const int zc = (v.nz + nzb - 1) / nzb;            // slices per pass, even split
    const dim3 grid((v.nx + kBpTileX - 1) / kBpTileX, (v.ny + kBlock / kBpTileX - 1) / (kBlock / kBpTileX),
                    (v.nz + zc - 1) / zc);
    if (grid.y > 65535 || grid.z > 65535) return hipErrorInvalidValue;
    if (!filt) {
#define FCAT_BP_CASE(Z)                                                                                      \
    case Z:                                                                                                  \
        hipLaunchKernelGGL(k_fdk_backproject<Z>, grid, dim3(kBlock), 0, stream, g, v, quads, cs, n, weight,  \
                           accumulate, volume);                                                              \
        break;
        switch (zc) {
            FCAT_BP_CASE(1) FCAT_BP_CASE(2) FCAT_BP_CASE(3) FCAT_BP_CASE(4) FCAT_BP_CASE(5) FCAT_BP_CASE(6)
            FCAT_BP_CASE(7) FCAT_BP_CASE(8) FCAT_BP_CASE(9) FCAT_BP_CASE(10) FCAT_BP_CASE(11) FCAT_BP_CASE(12)
            FCAT_BP_CASE(13) FCAT_BP_CASE(14) FCAT_BP_CASE(15) FCAT_BP_CASE(16)
        default: return hipErrorInvalidValue;
        }
#undef FCAT_BP_CASE
    } else
        hipLaunchKernelGGL(k_fdk_backproject_dense, grid, dim3(kBlock), 0, stream, g, v, filt, cs, n, zc, weight,
                           accumulate, volume);
    return hipGetLastError();
}

}  // namespace fcat
