// Internal declarations shared by the C-ABI layer and the gfx950 kernels of
// libfcat.so.  Not part of the public interface (include/fcat.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/fcat.h"

namespace fcat {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per workgroup (4 waves)
constexpr int kXcds = 8;           // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kBrickEdge = 16;     // edge of the cubic label bricks of the two-level walk (8 and 32 measured slower)
constexpr int kBrickVox = kBrickEdge * kBrickEdge * kBrickEdge;
// Padding before and after the brick-major labels, filled with 0xFF (a label
// that only ever reaches the spare accumulator slot).  Inside a brick the
// voxel walk takes at most 3 kBrickEdge + 4 steps of at most kBrickEdge^2
// bytes each, so a walk that rounding carries past the brick face reads
// padding or a neighbouring brick, never outside the buffer: no clamp of
// the offset is needed per step.
constexpr uint32_t kLabelPad = 16384;
static_assert(kLabelPad >= (3 * kBrickEdge + 4) * kBrickEdge * kBrickEdge, "label padding covers the walk");

// Ray geometry of one launch, everything a lane needs to build its ray in
// FP64.  lo/h/n describe the voxel grid; cu/cv are the detector centre
// indices (N-1)/2.
struct TraceGeom {
    double sid, back;              // SID and SDD - SID
    double du, dv, off_u, off_v;
    double cu, cv;
    double lo[3], h[3], inv_h[3];
    int n[3];
    int nu, nv, n_angles;
    const double *angles;          // device, or null for 2 pi a / A
    const double *trig;            // device [n_angles][2]: cos, sin of each angle, or null
    // Brick map of the labels: kBrickEdge^3 bricks, nb[] per axis; bricks[]
    // ([nb2][nb1][nb0]) holds the common label of a uniform brick or -1, and
    // labels_bm[brick][z][y][x] is the brick-major copy of the labels, with
    // kLabelPad bytes of padding before brick 0 and after the last brick.
    int nb[3];
    const int8_t *bricks;
    const int8_t *labels_bm;
    // The background box (device int[8], or null): every voxel outside the
    // voxel box [clip[1..3], clip[4..6]) holds label clip[0]; clip[7] is 0 when
    // the box is empty (the whole grid holds clip[0]).  The walk starts and
    // ends at this box and charges the rest of the ray to clip[0] in one sum.
    const int *clip;
    // Detector pixels of one wavefront: a (1 << tile_log2u) x (64 >> tile_log2u)
    // tile (columns x rows) of one angle.  Compact tiles keep the 64 rays of a
    // wavefront close in space, so they cross the same bricks at nearly the
    // same steps (far less divergence than 64 pixels of one row).
    int tile_log2u;
    // Input problems found while reading the inputs, or null: bad[0] |= 1 for
    // a label outside 0..n_mat-1, bad[1] |= 1 for a non-finite table value.
    int *bad;
};

// Input-problem flags at the start of a projector workspace: [0] label out
// of range, [1] non-finite table value.
constexpr int kInputFlags = 2;

// Where the preparation kernels report input problems (see TraceGeom::bad):
// psf kernels (n_psf floats) are checked beside the spectral tables.
struct InputCheck {
    const float *psf = nullptr;
    int n_psf = 0;
    int *bad = nullptr;
};

// Tile shape for a geometry: 8 x 8 pixels, or 16 x 4 where the phantom
// covers only a few detector rows (a thin slab), so that fewer lanes of a
// wavefront fall outside it.
int tile_log2u_for(const TraceGeom &G);
inline int64_t tiles_per_angle_host(const TraceGeom &G)
{
    const int tu = 1 << G.tile_log2u, tv = kWave >> G.tile_log2u;
    return (int64_t)((G.nu + tu - 1) / tu) * ((G.nv + tv - 1) / tv);
}

// Workgroups of a launch with one wavefront per tile of detector pixels,
// padded to a multiple of kXcds so that the XCD remap (xcd_block) is a
// bijection.
inline int padded_blocks(int64_t waves)
{
    const int64_t nblk = (waves + (kBlock / kWave) - 1) / (kBlock / kWave);
    return (int)((nblk + kXcds - 1) / kXcds * kXcds);
}

// Spectral tables prepared on the device (in the workspace) from mu, phi,
// eta and s_bin.  gstart is host-derived from the group map.
struct SpecTables {
    const float *muT;              // [E][mp]  (mp = padded material count, zeros past n_mat)
    const float *mu2T;             // [E][mp]  mu * log2(e), rounded once (optical depth in bits)
    const float *w;                // [E]      phi * eta
    const float *Wg;               // [G]      sum of w over the group
    const float *Wsg;              // [G]      sum of w * s_bin over the group
    int E, M, G, mp;
    int gstart[FCAT_MAX_GROUPS + 1];
};

// Tables of the split-precision contraction.  The energy axis is cut into
// tiles of 16 bins that never straddle two groups (each group is padded to a
// multiple of 16 bins with zero weight); tiles gtile[g] .. gtile[g+1]-1
// belong to group g.  afrag holds, per tile and 32-wide k block, the
// matrix-core A operand (16 energies x 32 k, BF16) in lane order: lane l has
// row l % 16 and k = 8 (l / 16) .. + 7.  k runs over [mu_hi | mu_lo | mu_hi]
// (n_mat each, zero-padded).  wtile[t][row] is phi * eta of the tile's bins.
struct SplitTables {
    const uint4 *afrag;            // [T][nkb][64]  (8 BF16 per lane)
    const float *wtile;            // [T][16]
    int T, nkb;
    int gtile[FCAT_MAX_GROUPS + 1];
};

// Surrogate network tables (fcat_mlp.hip).  frag holds the BF16 B-operand
// fragments of every weight view the forward and backward passes use.
constexpr int kMlpFrags = 69;
constexpr int kMlpTrainFrags = 40;
struct MlpTables {
    const uint4 *frag;             // [kMlpFrags][64]
    const float *params;           // FP32 master parameters (biases read from here)
    const float *in_scale;         // [n_in]
    const float *out_scale;        // [n_out]
    const float *lin;              // [n_out][n_in]
    const uint8_t *cell_ok;        // [n_in * FCAT_MLP_CELLS]
    const float *mbar;             // [n_in] spectrum-weighted mean attenuation per material
    float cell_lo, cell_hi;        // optical-depth range of the cells
    int n_in, n_out;
};

// Relative floor of the surrogate's error and loss weight: a group counts
// fully once it carries this share of the ray's primary signal.
constexpr float kMlpShareFloor = 1e-3f;
// Set-up statistics: fixed grid and per-block record of k_mlp_stats.
constexpr int kStatBlocks = 1024;
constexpr int kStatStride = 64;    // max L [16], max tau [1], sum w r^2 [16], sum w [16]

// Inputs and outputs of the surrogate spectral stage over n rays of L.
// Ray r belongs to angle r / plane, pixel r % plane.
struct SurrogateIO {
    const float *L;                // [n][n_mat]
    int64_t n, plane;
    const float *flood;            // [plane] or null
    const float *scatter;          // [n] or null
    float *Y;                      // [n / plane][G][plane] or null
    float *out;                    // [n] (sum over groups) or null
    int *counts;                   // [2]: rays by the network, rays by the exact sum; or null
    int force_mlp;                 // 1: no fallback (validation and training checks)
    int *bad;                      // bad[1] |= 1 for a non-finite flood or scatter value; or null
};

int mlp_param_count(int n_in, int n_out);
// BF16 fragment views of the network's weights: all kMlpFrags of them, or
// with training only the first kMlpTrainFrags (those the gradient kernel reads).
hipError_t launch_mlp_prep(const float *params, int n_in, int n_out, uint4 *frag, hipStream_t stream,
                           bool training = false);
hipError_t launch_mlp_linear(const float *mu, const SpecTables &t, float *lin, hipStream_t stream);
hipError_t launch_mlp_mbar(const SpecTables &t, const float *lin, float *mbar, hipStream_t stream);
hipError_t launch_mlp_stats(const SpecTables &t, const float *lin, const float *mbar, const float *L, const float *Y,
                            int64_t n, float *partial, float *in_scale, float *out_scale, float *tau_max,
                            hipStream_t stream);
hipError_t launch_mlp_spectral(const SpecTables &t, const MlpTables &m, const SurrogateIO &io, hipStream_t stream);
// Ray counts of the surrogate projector: wavefront gw adds its two counts
// (rays by the network, rays by the exact sum) to the first two ints of slot
// gw % kCountSlots, one 64-byte line per slot, so that no address takes more
// than a small share of the adds (adds from every wavefront to one address
// took 3 ms per launch of 16 head angles); launch_count_slots_sum adds the
// slots' totals to the caller's two counters.
constexpr int kCountSlots = 512;
constexpr int kCountSlotInts = 16;
// The surrogate projector for angles [a0, a0 + n_ang) in one pass (walk,
// network where validated, exact sum elsewhere, scatter); Y and out as in
// launch_project_rows; slots: kCountSlots * kCountSlotInts ints, zero before
// the first launch of a call, or null.
hipError_t launch_project_rows_mlp(const TraceGeom &g, const SpecTables &t, const MlpTables &m, const float *flood,
                                   const float *scatter, int a0, int n_ang, float *Y, float *out, int *slots,
                                   hipStream_t stream);
hipError_t launch_count_slots_sum(const int *slots, int *counts, hipStream_t stream);
hipError_t launch_mlp_grad(const SpecTables &t, const MlpTables &m, const float *L, const float *Y, int64_t n_all,
                           const int32_t *order, int64_t base, int count, float *partial, float *loss_partial,
                           hipStream_t stream);
// With cnt and inv (from launch_mlp_frag_inverse) the Adam step also rewrites, in
// frag, the training fragment elements of every parameter it updates.
hipError_t launch_mlp_reduce_adam(const float *partial, int nparts, int P, float *grad, float *params, float *m,
                                  float *v, int step, float lr, float beta1, float beta2, float eps,
                                  const float *loss_partial, float loss_scale, float *loss_out, hipStream_t stream,
                                  const int *cnt = nullptr, const uint32_t *inv = nullptr, uint4 *frag = nullptr);
// Elements of the training fragments per parameter: up to kMlpViews entries
// per parameter in inv ([P][kMlpViews]), their number in cnt ([P] ints).
constexpr int kMlpViews = 4;
hipError_t launch_mlp_frag_inverse(int n_in, int n_out, int *cnt, uint32_t *inv, hipStream_t stream);
hipError_t launch_mlp_validate(const SpecTables &t, const MlpTables &m, const float *L, const float *Y, int64_t n,
                               unsigned *err_bits, int *count, hipStream_t stream);
hipError_t launch_mlp_cells(const unsigned *err_bits, const int *count, int ncell, float threshold, int min_count,
                            float *cell_err, uint8_t *cell_ok, hipStream_t stream);

// Launch helpers (fcat_kernels.hip).  All are stream-ordered and return the
// hipError_t of the launch.
hipError_t launch_prep_tables(const float *mu, const float *phi, const float *eta,
                              const float *s_bin, const SpecTables &t, float *muT, float *w,
                              float *Wg, float *Wsg, hipStream_t stream, const InputCheck &chk = InputCheck());

// Fused traversal + spectral sum for angles [a0, a0 + n_ang).  When Y is
// non-null the group signals go to Y[a - a0][g][v][u]; otherwise
// out[a][v][u] receives their sum.
hipError_t launch_project_rows(const TraceGeom &g, const int8_t *labels, const SpecTables &t,
                               const float *flood, const float *scatter, int a0, int n_ang,
                               float *Y, float *out, hipStream_t stream);

// Fills trig[2 a], trig[2 a + 1] with the cosine and sine of every angle of g.
hipError_t launch_trig_table(const TraceGeom &g, double *trig, hipStream_t stream);

// Builds SplitTables::afrag and ::wtile from mu and the prepared w.
hipError_t launch_prep_split(const float *mu, const SpecTables &t, const SplitTables &sp, uint4 *afrag,
                             float *wtile, hipStream_t stream);

// Same as launch_project_rows with the L . mu contraction on matrix cores
// (BF16 hi/lo split, FP32 accumulate).
hipError_t launch_project_rows_split(const TraceGeom &g, const int8_t *labels, const SpecTables &t,
                                     const SplitTables &sp, const float *flood, const float *scatter, int a0,
                                     int n_ang, float *Y, float *out, hipStream_t stream);

// Brick map and brick-major label copy (see TraceGeom::bricks).
// Also writes the background box (see TraceGeom::clip) to clip (int[8]).
hipError_t launch_build_bricks(const int8_t *labels, int nx, int ny, int nz, int8_t *bricks, int8_t *labels_bm,
                               int *clip, hipStream_t stream, int n_mat = 0, int *bad = nullptr);

hipError_t launch_pathlengths(const TraceGeom &g, const int8_t *labels, int n_mat, int a0,
                              int n_ang, float *L, hipStream_t stream);
// Step counts of the walk (see fcat_walk_stats); counts must be zero first.
constexpr int kWalkCounts = 6;
hipError_t launch_walk_stats(const TraceGeom &g, int a0, int n_ang, unsigned long long *counts, hipStream_t stream);

// Projector of a voxel image and its transpose (fcat_adjoint.hip): the grid
// is described by g's lo/h/n; proj is [n_ang][nv][nu] for angles a0 ..
// a0 + n_ang - 1; the back-projection adds into image (zero it first for A^T y).
hipError_t launch_image_project(const TraceGeom &g, const float *image, int a0, int n_ang, float *proj,
                                hipStream_t stream);
hipError_t launch_image_backproject(const TraceGeom &g, const float *proj, int a0, int n_ang, float *image,
                                    hipStream_t stream);

hipError_t launch_spectral(const float *L, int64_t n, const SpecTables &t, const float *i0,
                           const float *S, float *Y, hipStream_t stream);
hipError_t launch_spectral_split(const float *L, int64_t n, const SpecTables &t, const SplitTables &sp,
                                 const float *i0, const float *S, float *Y, hipStream_t stream);

hipError_t launch_psf(const float *Y, int n_ang, int G, int nv, int nu, const float *kernels,
                      int k, float *out, hipStream_t stream);
// A Richardson-Lucy step fused into a one-group convolution (k = 15 only):
// step 1 writes out = c > 0 ? data / c : 0, step 2 writes out = out c / norm
// (norm one plane [nv][nu]), where c is the convolution of Y with kernel.
hipError_t launch_psf_rl(int step, const float *Y, int n_ang, int nv, int nu, const float *kernel, int k,
                         float *out, const float *data, const float *norm, hipStream_t stream);

// Optical spread of the split form on the matrix cores (BF16 hi/lo, FP32
// accumulate), for odd k <= kPsfSplitMaxK: B fragments of the banded kernel
// rows (G * k * 2 * 64 uint4), then the convolution and group sum.
constexpr int kPsfSplitMaxK = 17;
inline size_t psf_split_frag_count(int G, int k) { return (size_t)G * k * 2 * kWave; }
hipError_t launch_prep_psf_split(const float *kernels, int G, int k, uint4 *frag, hipStream_t stream);
hipError_t launch_psf_split(const float *Y, int n_ang, int G, int nv, int nu, int k, const uint4 *frag, float *out,
                            hipStream_t stream);

// Noise and projection stage (fcat_noise.hip).  Poisson counts on the
// group signals of n_ang angles (Y [n_ang][G][plane], in place), the count
// scale of Eq. 5 per group, the flood's group signals W_g I0, and
// proj = -ln(max(out, floor) / flood).
hipError_t launch_poisson(float *Y, int n_ang, int G, int64_t plane, const float *scale, uint64_t seed,
                          int angle_base, hipStream_t stream);
hipError_t launch_count_scale(const float *phi, const float *eta, const int *gstart, int E, int G, double H,
                              float *scale, hipStream_t stream);
hipError_t launch_flood_groups(const float *Wg, const float *i0, int64_t plane, int G, float *Yf, hipStream_t stream);
hipError_t launch_log_projection(const float *out, const float *flood, int n_ang, int64_t plane, float floor_,
                                 float *proj, hipStream_t stream);
hipError_t launch_fill(float *x, int n, float v, hipStream_t stream);

// Dose estimate (fcat_dose.hip).  Per chunk of rays with path lengths L
// [n_rays][M]: partial sums of 1 - exp(-P) per workgroup and energy bin
// (dose_blocks(n_rays) x E doubles), then S[e] += their sum in a fixed order;
// finally D0 and Dp from S.
// A prime, so that the tiles of a workgroup (stride kDoseBlocks) move across
// the positions of a detector row from one visit to the next: rays that meet
// the phantom come in bands of rows, and a stride that is a multiple of the
// row period would hand them all to a few workgroups.
constexpr int kDoseBlocks = 2039;
int dose_blocks(int64_t n_rays);
hipError_t launch_dose_rays(const float *L, int64_t n_rays, int M, const SpecTables &t, double *partial,
                            hipStream_t stream);
hipError_t launch_dose_sum(const double *partial, int nblk, int E, double *S, hipStream_t stream);
hipError_t launch_dose_final(const double *S, const float *energy, const float *ratio, const float *phi, int E,
                             double inv_nm, double *D0, double *Dp, hipStream_t stream);
hipError_t launch_zero_doubles(double *x, int n, hipStream_t stream);

hipError_t launch_check_labels(const int8_t *labels, int64_t n, int n_mat, int *flag,
                               hipStream_t stream);
hipError_t launch_check_finite(const float *x, int64_t n, int *flag, hipStream_t stream);
hipError_t launch_zero_ints(int *p, int n, hipStream_t stream);

}  // namespace fcat
