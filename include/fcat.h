/*
 * fcat -- polyenergetic cone-beam projector for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libfcat.so.  The projector computes, for every projection angle
 * and detector pixel, the fastCAT detected signal (O'Connell and
 * Bazalova-Carter, "FastCAT: Fast Cone Beam CT (CBCT) Simulation",
 * arXiv 2011.04736):
 *
 *   L_m      = length of the source-to-pixel-centre ray inside material m
 *              (Sec. II.F: a projection is the line integral of the
 *              attenuation along the ray; Sec. II.C: the phantom is an array
 *              of integer material labels 0..n-1, so mu(E, x) = mu_label(x)(E));
 *   P_e      = sum_m mu[m][e] L_m                        (one projection per energy, Sec. II.F)
 *   Y_g      = sum_{e in group g} phi_e eta_e (I0 exp(-P_e) + s_e S)
 *              (Eq. 3, with the scatter map S added to the primary intensity
 *              profiles before the spectrum x response weighting, Sec. II.F)
 *   out      = sum_g K_g (*) Y_g                         (Sec. II.G: each profile is
 *              convolved with its optical spread function, Eq. 1, and summed)
 *
 * Geometry conventions (the paper fixes none of them; these are this
 * library's): world z is the rotation axis and the isocentre is the origin;
 * the source is at (SID cos t, SID sin t, 0); the detector centre at
 * -(SDD - SID)(cos t, sin t, 0); the detector u axis is (-sin t, cos t, 0)
 * and v axis (0, 0, 1); pixel (iv, iu) has its centre at
 * c + ((iu - (Nu-1)/2) du + off_u) u + ((iv - (Nv-1)/2) dv + off_v) v;
 * t_a = 2 pi a / A unless explicit angles are given.  Voxel (ix, iy, iz) is
 * the half-open box [x0 + ix dx, x0 + (ix+1) dx) x ... with
 * x0 = cx - Nx dx / 2.  Lengths are in mm, attenuation in mm^-1.
 *
 * Memory and ordering rules for every entry point:
 *  - Descriptors are host structs, read during the call only.
 *  - Every array pointer is caller-owned DEVICE memory unless its comment
 *    says HOST.  The library never allocates, frees or retains device
 *    memory; scratch comes only from the caller's workspace (256-byte
 *    aligned, at least the size the matching *_workspace_bytes returns).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream)
 *    and is asynchronous with respect to the host, except fcat_check_inputs,
 *    which synchronises its stream.  Calls on different streams must use
 *    different workspaces.
 *  - Arguments are validated on the host before anything is launched; on a
 *    non-OK status nothing has been enqueued and outputs are untouched.
 *    fcat_last_error() then gives a description.  Device-side failures of
 *    earlier work surface as FCAT_E_DEVICE from a later call.
 *  - Labels outside 0..n_mat-1 are never used as an index: such voxels add
 *    no path length to any material.  Non-finite inputs are used as given
 *    (a NaN in mu makes the output of every ray that meets the phantom NaN,
 *    since the contraction multiplies it by each path length, zero or not).  fcat_project and fcat_projections note both while they read
 *    their inputs, without synchronising; fcat_project_status reports what
 *    the last such call found.  fcat_check_inputs checks them up front.
 */
#ifndef FCAT_H
#define FCAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCAT_VERSION 1

/* The enumerations below are 32-bit integers at the interface.  C++ gives
   them that fixed underlying type, so that every value a C caller passes
   (also one that names no enumerator) is a value of the type and is
   rejected or reported as unknown, not undefined. */
#ifdef __cplusplus
#define FCAT_ENUM_INT : int32_t
#else
#define FCAT_ENUM_INT
#endif

/* Largest supported sizes. */
#define FCAT_MAX_MATERIALS 32   /* n_mat */
#define FCAT_MAX_GROUPS 32      /* n_groups */
#define FCAT_MAX_ENERGIES 4096  /* n_energy */
#define FCAT_MAX_PSF 31         /* psf k (odd) */

typedef enum fcat_status FCAT_ENUM_INT {
    FCAT_OK = 0,
    FCAT_E_INVALID_ARG = 1,  /* null pointer, bad size, SDD <= SID, even k, bad group map ... */
    FCAT_E_WORKSPACE = 2,    /* workspace missing, misaligned or too small */
    FCAT_E_LABEL_RANGE = 3,  /* a label is outside 0..n_mat-1 (fcat_project_status, fcat_check_inputs) */
    FCAT_E_NONFINITE = 4,    /* NaN or Inf in a float input (fcat_project_status, fcat_check_inputs) */
    FCAT_E_DEVICE = 5,       /* a HIP runtime error (text in fcat_last_error) */
    FCAT_E_UNSUPPORTED = 6   /* a valid request this library does not implement */
} fcat_status;

typedef enum fcat_mode FCAT_ENUM_INT {
    FCAT_MODE_PLAIN = 0,       /* FP32 traversal and FP32 spectral sum */
    FCAT_MODE_SPLIT_BF16 = 1,  /* L . mu on matrix cores, BF16 hi/lo split, FP32 accumulate */
    FCAT_MODE_SURROGATE = 2    /* learned per-group attenuation with exact fallback */
} fcat_mode;

/* Circular cone-beam geometry (Sec. II: SAD 1.00 m, SDD 1.52 m by default). */
typedef struct fcat_geometry_t {
    double sid_mm;            /* source to isocentre, > 0 */
    double sdd_mm;            /* source to detector, > sid_mm */
    int32_t nu, nv;           /* detector columns (u, fastest) and rows, >= 1 */
    double du_mm, dv_mm;      /* pixel pitch, > 0 */
    double off_u_mm, off_v_mm;/* detector shift along u and v */
    int32_t n_angles;         /* >= 1 */
    const double *angles_rad; /* DEVICE [n_angles] radians, or NULL for 2 pi a / n_angles (device
                                 memory so that every lane reads its angle where it builds its ray) */
} fcat_geometry_t;

/* Labelled voxel phantom (Sec. II.C). */
typedef struct fcat_phantom_t {
    int32_t nx, ny, nz;       /* >= 1 each */
    double dx_mm, dy_mm, dz_mm;
    double cx_mm, cy_mm, cz_mm; /* centre of the grid */
    const int8_t *labels;     /* DEVICE [nz][ny][nx], x fastest */
} fcat_phantom_t;

/* Attenuation tables, spectrum and detector response (Sec. II.A-C, Eq. 3). */
typedef struct fcat_spectral_t {
    int32_t n_mat;            /* 1..FCAT_MAX_MATERIALS */
    int32_t n_energy;         /* 1..FCAT_MAX_ENERGIES */
    int32_t n_groups;         /* 1..min(n_energy, FCAT_MAX_GROUPS) */
    const float *mu;          /* DEVICE [n_mat][n_energy], mm^-1 */
    const float *phi;         /* DEVICE [n_energy] fluence spectrum */
    const float *eta;         /* DEVICE [n_energy] energy deposition efficiency */
    const float *flood;       /* DEVICE [nv][nu] flood intensity I0, or NULL for 1 */
    const int32_t *group_of_bin; /* HOST [n_energy], non-decreasing, each group non-empty,
                                    or NULL for floor(e * n_groups / n_energy); host memory
                                    because it is validated and turned into group bounds on the
                                    host before anything is launched */
} fcat_spectral_t;

/* Pre-tabulated scatter (Sec. II.E), added to the primary profiles. */
typedef struct fcat_scatter_t {
    const float *maps;        /* DEVICE [n_angles][nv][nu] */
    const float *s_bin;       /* DEVICE [n_energy] per-bin scale, or NULL for 1 */
} fcat_scatter_t;

/* Optical spread kernels per energy group (Eq. 1, Sec. II.G). */
typedef struct fcat_psf_t {
    int32_t k;                /* odd, 1..FCAT_MAX_PSF */
    const float *kernels;     /* DEVICE [n_groups][k][k]; out = sum_g K_g (*) Y_g, true
                                 convolution, zero outside the detector, centre (k-1)/2 */
} fcat_psf_t;

/*
 * Learned replacement of the primary spectral sum (MLP with SiLU).
 * For a ray with path lengths L (n_in = n_mat values):
 *   x_m  = L_m * in_scale[m]
 *   z_g  = sum_m lin[g][m] L_m + out_scale[g] MLP(x)_g
 *   Y_g  = I0 W_g exp(-z_g) + Ws_g S          with W_g = sum_{e in g} phi_e eta_e
 * MLP: h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2), MLP(x) = W3 h2 + b3.
 * Every product a.b runs on the matrix cores as a_hi.b_hi + a_lo.b_hi +
 * a_hi.b_lo with a_hi = bf16(a), a_lo = bf16(a - a_hi), FP32 accumulation.
 *
 * Validated domain.  With mbar_m = sum_e phi_e eta_e mu[m][e] / sum_e phi_e eta_e
 * (the spectrum-weighted mean attenuation), the cell of a hit ray is
 * (argmax_m mbar_m L_m) * 16 + floor(16 (tau - cell_lo) / (cell_hi - cell_lo)),
 * tau = sum_m mbar_m L_m its mean optical depth.  The exact spectral sum is
 * used wherever the ray misses, some x_m > 1, tau is outside
 * [cell_lo, cell_hi), or cell_ok[cell] is 0.  fcat_project takes the network
 * only for groups of 64 neighbouring rays (one wavefront: an 8 x 8 or 16 x 4
 * tile of detector pixels of one angle) whose hit rays all lie in the
 * domain, and the exact sum for every ray of the other groups.
 */
#define FCAT_MLP_HIDDEN 64
#define FCAT_MLP_CELLS 16
#define FCAT_MLP_MAX_IO 16
#define FCAT_MLP_MAX_BATCH 65536
typedef struct fcat_surrogate_t {
    int32_t n_in;             /* == n_mat, 1..16 */
    int32_t n_out;            /* == n_groups, 1..16 */
    const float *params;      /* DEVICE FP32 [fcat_mlp_param_count]: W1[64][n_in], b1[64],
                                 W2[64][64], b2[64], W3[n_out][64], b3[n_out] */
    const float *in_scale;    /* DEVICE [n_in] */
    const float *out_scale;   /* DEVICE [n_out] */
    const float *lin;         /* DEVICE [n_out][n_in] (fcat_mlp_linear_term) */
    const uint8_t *cell_ok;   /* DEVICE [n_in * 16] (fcat_mlp_validate); needed by fcat_project only */
    float cell_lo, cell_hi;   /* optical-depth range of the 16 bins, cell_lo < cell_hi */
    int32_t *counts;          /* DEVICE [2] or NULL: fcat_project adds the number of rays the
                                 network handled and the number that fell back to the exact sum */
} fcat_surrogate_t;

/* Training state of the surrogate (Adam, Kingma & Ba 2015). */
typedef struct fcat_mlp_train_t {
    float *params;            /* DEVICE FP32 [P], updated in place */
    float *adam_m, *adam_v;   /* DEVICE FP32 [P], zero before the first step */
    int32_t step;             /* Adam steps taken so far; each update increments it */
    float lr, beta1, beta2, eps;
} fcat_mlp_train_t;

/* ---------------------------------------------------------------- status */

/* Static description of a status code. */
const char *fcat_status_string(fcat_status s);
/* Detail of the last non-OK status returned on the calling thread ("" if none). */
const char *fcat_last_error(void);
/* FCAT_VERSION of the built library. */
int fcat_version(void);

/* ------------------------------------------------------------ projector */

/*
 * Workspace needed by fcat_project.  angles_per_chunk = 0 lets the library
 * choose: every angle in one chunk if their group signals fit in 1 GiB,
 * else chunks of at most 384 MiB of them.  fcat_project processes as many angles per chunk as the workspace
 * it is given holds.  Returns 0 if the descriptors are invalid.
 */
size_t fcat_project_workspace_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                    const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                                    const fcat_psf_t *psf, fcat_mode mode, int32_t angles_per_chunk);

/*
 * Full projector: out[a][v][u] (DEVICE float [n_angles][nv][nu]) for every
 * angle and pixel.  scatter NULL turns the scatter term off; psf NULL turns
 * the optical spread off (out = sum_g Y_g).  surrogate is required for
 * FCAT_MODE_SURROGATE and ignored otherwise; in that mode one kernel walks
 * each ray, evaluates the network on the matrix cores for the rays whose
 * cell is validated and takes the exact spectral sum for the others (path
 * lengths stay in registers).
 */
fcat_status fcat_project(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                         const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                         const fcat_psf_t *psf, fcat_mode mode, const fcat_surrogate_t *surrogate,
                         float *out, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Input problems found by the last fcat_project or fcat_projections call that
 * used `workspace` (the same pointer, on the same stream): labels outside
 * 0..n_mat-1 (FCAT_E_LABEL_RANGE, checked first: Sec. II.C numbers the
 * materials 0..n-1) and non-finite values in mu, phi, eta, s_bin, flood, the
 * scatter maps or the spread kernels (FCAT_E_NONFINITE).  The projector call
 * itself returns as soon as its work is enqueued, so it cannot know; its
 * kernels set two flags at the start of the workspace as they read each
 * input (the labels when the brick map is built, the tables when they are
 * prepared, flood and scatter where each ray reads them), after clearing
 * them at the start of the call.  This call waits for the stream
 * (hipStreamSynchronize) and reads the flags; it launches nothing and
 * changes nothing.  Returns FCAT_OK when none is set.
 */
fcat_status fcat_project_status(const void *workspace, size_t workspace_bytes, void *stream);

/* Workspace needed by fcat_pathlengths (the brick map of the labels). */
size_t fcat_pathlengths_workspace_bytes(const fcat_phantom_t *phantom);

/*
 * Per-material path lengths (Sec. II.F line integral, Sec. II.C labels) of
 * every pixel of angles a_begin <= a < a_end:
 * L = DEVICE float [a_end - a_begin][nv][nu][n_mat].
 */
fcat_status fcat_pathlengths(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                             int32_t n_mat, int32_t a_begin, int32_t a_end, float *L, void *workspace,
                             size_t workspace_bytes, void *stream);

/*
 * Work the exact walk does for the rays of angles a_begin <= a < a_end, for
 * cost models and roofline accounting (the projector's own walk, counting
 * instead of charging lengths).  counts (DEVICE int64 [6], overwritten):
 *   [0] rays that meet the grid,
 *   [1] brick steps (uniform bricks cross in one step each),
 *   [2] mixed bricks entered,
 *   [3] voxel steps inside mixed bricks,
 *   [4] lane slots of the voxel loop: its wavefront iterations times 64
 *       (one lane follows one ray; a wavefront iterates until its slowest
 *       lane is done, so [4] / [3] measures the divergence),
 *   [5] voxel segments of Siddon's method: per ray that meets the grid,
 *       1 + sum over axes of |i_exit - i_entry| (entry and exit voxels by
 *       floor of the FP64 entry and exit points).
 * Siddon's method (Sec. II.F's line integral through the labelled phantom)
 * steps once per voxel segment, [5]; [1] + [3] is what this walk takes.
 * Workspace: fcat_pathlengths_workspace_bytes(phantom) bytes.
 */
fcat_status fcat_walk_stats(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom, int32_t a_begin,
                            int32_t a_end, int64_t *counts, void *workspace, size_t workspace_bytes, void *stream);

/* Workspace needed by fcat_spectral. */
size_t fcat_spectral_workspace_bytes(const fcat_spectral_t *spectral);

/*
 * Eq. 3 for a list of rays: Y[g][r] (DEVICE float [n_groups][n]) from
 * L (DEVICE float [n][n_mat]).  i0 (DEVICE [n]) NULL means 1; S (DEVICE [n])
 * NULL means no scatter; s_bin (DEVICE [n_energy]) NULL means 1.
 * spectral->flood is ignored (pass i0).  mode PLAIN or SPLIT_BF16.
 */
fcat_status fcat_spectral(const float *L, int64_t n, const fcat_spectral_t *spectral,
                          const float *i0, const float *S, const float *s_bin, fcat_mode mode,
                          float *Y, void *workspace, size_t workspace_bytes, void *stream);

/*
 * fcat_spectral without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as fcat_spectral;
 * its tables (at most about 1.4 MiB: n_energy <= 4096, n_mat <= 32) go to a
 * static 2 MiB device array of the library, which each GPU it runs on holds
 * from the first call until the process ends.  The call allocates nothing.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (different streams, threads) race and must not be made; calls
 * on one stream are ordered and safe.  Tables larger than the array give
 * FCAT_E_UNSUPPORTED (none within the limits above does).
 */
fcat_status fcat_spectral_static(const float *L, int64_t n, const fcat_spectral_t *spectral,
                                 const float *i0, const float *S, const float *s_bin, fcat_mode mode,
                                 float *Y, void *stream);

/*
 * Optical spread and group sum (Sec. II.G): out[a][v][u] =
 * sum_g sum_{p,q} K[g][p][q] Y[a][g][v-p+c][u-q+c], zero outside, c = (k-1)/2.
 * Y DEVICE float [n_ang][n_groups][nv][nu], out DEVICE float [n_ang][nv][nu].
 */
fcat_status fcat_psf(const float *Y, int32_t n_ang, int32_t n_groups, int32_t nv, int32_t nu,
                     const fcat_psf_t *psf, float *out, void *stream);

/*
 * Device-data validation (synchronises `stream`): labels in 0..n_mat-1 and
 * every float table finite.  Any descriptor but phantom and spectral may be
 * NULL.  Needs 256 bytes of workspace.  Returns FCAT_E_LABEL_RANGE or
 * FCAT_E_NONFINITE on a violation.
 */
fcat_status fcat_check_inputs(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                              const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                              const fcat_psf_t *psf, void *workspace, size_t workspace_bytes,
                              void *stream);

/* ------------------------------------------------- noise and projections */
/*
 * Sec. II.G, Eq. 5.  Noise is a Poisson scaling of the counts on the
 * detector, with the flood field scaled to a height of H counts per pixel
 * (H = N_gamma / (A / A_p): particles over beam area in pixel areas); the
 * scatter takes Poisson noise from its pixel's counts; the noisy profiles go
 * through the optical spread and the group sum and come back as projections
 * through the flood field.  The paper leaves the details open; this library
 * computes:
 *   c_g    = H Phi_g / (Phi W_g)          count scale of group g, with
 *            Phi_g = sum_{e in g} phi_e, Phi = sum_e phi_e, W_g = sum_{e in g} phi_e eta_e
 *            (FP64 sums in bin order, rounded to float; 0 if Phi_g or W_g is 0),
 *            so an open pixel with I0 = 1 holds H Phi_g / Phi photons of group g
 *            and H in all;
 *   Y_g   <- n / c_g,  n ~ Poisson(float(c_g * Y_g))   (before the spread; n / c_g
 *            in FP32 to 2 ulp; the scatter inside Y_g needs no draw of its own,
 *            a sum of independent Poisson counts being Poisson; a group with
 *            c_g <= 0 passes unchanged);
 *   flood  = sum_g K_g (*) (W_g I0)       noiseless, object-free, no scatter;
 *   proj   = -ln(max(out, floor) / flood).
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), key
 * (seed mod 2^32, seed div 2^32), counters (pixel, group, angle, j) for
 * j = 0, 1, ..., each block giving the pairs (u, v) = (w0, w1), (w2, w3) as
 * (w + 1/2) 2^-32.  Pixel is v * nu + u, angle the index in the full scan.
 * Poisson variates: for a mean below 16, the smallest k with u <= F(k) (CDF
 * summed term by term, at most 256 terms); otherwise the transformed
 * rejection method PTRS (Hormann 1993), one pair per attempt, at most 64
 * attempts (then floor(mean + 1/2)); FP64 throughout.  A draw therefore
 * depends only on (seed, pixel, group, angle, mean), never on launch shape,
 * chunking or stream.
 */
typedef struct fcat_noise_t {
    double counts_per_pixel;  /* H of Eq. 5, > 0 */
    uint64_t seed;            /* Philox key */
    float floor;              /* >= 0: lower bound of the detected profile before the log;
                                 0 lets a pixel with no counts give +inf */
} fcat_noise_t;

/* c_g of Eq. 5 (see above) into scale (DEVICE float [n_groups]). */
fcat_status fcat_count_scale(const fcat_spectral_t *spectral, double counts_per_pixel, float *scale, void *stream);

/*
 * Poisson noise on group signals, in place: Y (DEVICE float
 * [n_ang][n_groups][plane]) holds angles angle_base .. angle_base + n_ang - 1;
 * scale is DEVICE float [n_groups].  plane < 2^31, angle_base >= 0.
 */
fcat_status fcat_poisson(float *Y, int32_t n_ang, int32_t n_groups, int64_t plane, const float *scale,
                         uint64_t seed, int32_t angle_base, void *stream);

/* Workspace needed by fcat_flood_profile. */
size_t fcat_flood_workspace_bytes(const fcat_spectral_t *spectral, int32_t nv, int32_t nu);

/*
 * Noiseless object-free flood through the spread: flood (DEVICE float
 * [nv][nu]) = sum_g K_g (*) (W_g I0), I0 = spectral->flood (NULL: 1).
 * psf NULL gives sum_g W_g I0.
 */
fcat_status fcat_flood_profile(const fcat_spectral_t *spectral, const fcat_psf_t *psf, int32_t nv, int32_t nu,
                               float *flood, void *workspace, size_t workspace_bytes, void *stream);

/*
 * proj[a][p] = -ln(max(out[a][p], floor) / flood[p]) for out, proj DEVICE
 * float [n_ang][plane] (proj may equal out) and flood DEVICE float [plane].
 */
fcat_status fcat_log_projection(const float *out, const float *flood, int32_t n_ang, int64_t plane, float floor,
                                float *proj, void *stream);

/* Workspace needed by fcat_projections (arguments as for fcat_project_workspace_bytes). */
size_t fcat_projections_workspace_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                        const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                                        const fcat_psf_t *psf, fcat_mode mode, int32_t angles_per_chunk);

/*
 * The projector followed by the noise and projection stage:
 * proj[a][v][u] (DEVICE float [n_angles][nv][nu]) = -ln(max(out, floor) / flood)
 * where out is fcat_project's detected profile with every group signal
 * replaced by its Poisson draw.  noise NULL gives noiseless projections
 * (floor 0).  Other arguments as for fcat_project.
 */
fcat_status fcat_projections(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                             const fcat_spectral_t *spectral, const fcat_scatter_t *scatter,
                             const fcat_psf_t *psf, fcat_mode mode, const fcat_surrogate_t *surrogate,
                             const fcat_noise_t *noise, float *proj, void *workspace, size_t workspace_bytes,
                             void *stream);

/* ------------------------------------------------------------------ dose */
/*
 * Dose per particle (Sec. II.H, Eqs. 6-7) from the rays of angles
 * a_begin <= a < a_end, every detector pixel a ray (hit or not; N_i counts
 * them all):
 *   D0[e] = E_e (mu_en/mu)_e / (N_i M) sum_i (1 - exp(-P_i(e))),
 *           P_i(e) = sum_m mu[m][e] L_i,m  (the ray's projection; for a water
 *           phantom mu_water(E) x_i as in Eq. 6),
 *   Dp    = sum_e phi_e D0[e].
 * energy (E_e, any unit) and mu_en_over_mu ((mu_en/mu)_e of water, the
 * phantom's absorption standing in for the paper's water) are DEVICE float
 * [n_energy]; mass M > 0 in any unit: D0 is in energy units per mass unit
 * per particle.  D0 is DEVICE double [n_energy]; Dp DEVICE double [1] or
 * NULL.  Sums run in FP64 in a fixed order (deterministic for a given
 * workspace).  The paper's empirical fit to Monte Carlo doses, and the
 * number of particles a requested dose implies (dose / Dp, then Eq. 5 for
 * the noise), are left to the caller.
 */
size_t fcat_dose_workspace_bytes(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                                 const fcat_spectral_t *spectral, int32_t angles_per_chunk);
fcat_status fcat_dose(const fcat_geometry_t *geometry, const fcat_phantom_t *phantom,
                      const fcat_spectral_t *spectral, const float *energy, const float *mu_en_over_mu,
                      double mass, int32_t a_begin, int32_t a_end, double *D0, double *Dp, void *workspace,
                      size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------- reconstruction */
/*
 * FDK reconstruction of the circular scan (Sec. II.G: the projections are
 * reconstructed with the default FDK algorithm; Feldkamp, Davis and Kress,
 * J. Opt. Soc. Am. A 1 (1984) 612), in the geometry conventions above:
 *   virtual detector through the axis: a = u_det SID / SDD, c = v_det SID / SDD,
 *     pitch tau = du SID / SDD;
 *   q = p SID / sqrt(SID^2 + a^2 + c^2)                  (cosine weight)
 *   q~[n] = tau sum_k h((n - k) tau) q[k] along each row, zero beyond the
 *     detector, with the Ram-Lak kernel h(0) = 1/(4 tau^2), h(m tau) = 0 for
 *     even m != 0 and -1/(m^2 pi^2 tau^2) for odd m;
 *   f(x, y, z) = (pi / A) sum_a SID^2 / U^2 q~_a(a*, c*), with
 *     s = x cos b + y sin b, t = -x sin b + y cos b, U = SID - s,
 *     a* = SID t / U, c* = SID z / U, q~ sampled bilinearly (zero outside);
 *     A = n_angles and the scan is taken as a full, evenly spaced circle.
 * p is the line integral of attenuation (for instance fcat_projections'
 * output); f is then in mm^-1.  All FP32.
 */
typedef struct fcat_grid_t {
    int32_t nx, ny, nz;       /* >= 1 each, nx ny nz < 2^31 */
    double dx_mm, dy_mm, dz_mm;
    double cx_mm, cy_mm, cz_mm; /* centre; voxel i of an axis has its centre at c - n d / 2 + (i + 1/2) d */
} fcat_grid_t;

/*
 * Cosine weight and ramp filter: filtered (DEVICE float [n_ang][nv][nu]) from
 * proj (DEVICE float [n_ang][nv][nu]); the two must not overlap.
 * nu <= 7704 (a row and the filter taps are held in 64 KiB of LDS), else
 * FCAT_E_UNSUPPORTED.
 */
fcat_status fcat_fdk_filter(const fcat_geometry_t *geometry, const float *proj, int32_t n_ang, float *filtered,
                            void *stream);

/* Workspace needed by fcat_fdk_backproject for n_ang angles. */
size_t fcat_fdk_backproject_workspace_bytes(int32_t n_ang);

/*
 * Back-projection of filtered projections of angles a_begin .. a_end - 1
 * (DEVICE float [a_end - a_begin][nv][nu]) into volume (DEVICE float
 * [nz][ny][nx]): volume = (accumulate ? volume : 0) + (pi / n_angles) sum_a
 * (SID / U)^2 times the bilinear sample of the filtered rows at the voxel's
 * detector position (Sec. II.G; taps off the detector count as 0).  It
 * reads the caller's rows as they are; fcat_fdk, which lays its own filtered
 * rows out as zero-padded 2 x 2 sample quads, back-projects about 1.4x
 * faster.
 */
fcat_status fcat_fdk_backproject(const fcat_geometry_t *geometry, const float *filtered, int32_t a_begin,
                                 int32_t a_end, const fcat_grid_t *grid, float *volume, int32_t accumulate,
                                 void *workspace, size_t workspace_bytes, void *stream);

/*
 * Workspace needed by fcat_fdk: the angles' (cos, sin), then for each angle
 * of a chunk its filtered rows, zero-padded ((nv + 3) x max(nu, 2) floats),
 * and their 2 x 2 bilinear sample quads ((nv + 2) x (max(nu, 2) - 1)
 * float4); angles_per_chunk 0: as many angles as fit in 1 GiB.  A smaller
 * workspace than this makes fcat_fdk take fewer angles per chunk.
 */
size_t fcat_fdk_workspace_bytes(const fcat_geometry_t *geometry, int32_t angles_per_chunk);

/*
 * The whole reconstruction: volume (DEVICE float [nz][ny][nx]) from proj
 * (DEVICE float [n_angles][nv][nu]).  nu <= 7704 and
 * (nv + 2) (max(nu, 2) - 1) < 2^28, else FCAT_E_UNSUPPORTED.
 */
fcat_status fcat_fdk(const fcat_geometry_t *geometry, const float *proj, const fcat_grid_t *grid, float *volume,
                     void *workspace, size_t workspace_bytes, void *stream);

/*
 * The projector of a real-valued voxel image and its transpose, the pair an
 * iterative reconstruction alternates (Sec. II.F: a projection is the line
 * integral along the source-to-pixel ray; Sec. II.G: the projections are
 * reconstructed).  For the rays r of angles a_begin <= a < a_end (pixel
 * centres and angles as above) and the voxels k of grid (the phantom's
 * conventions: half-open boxes, image [nz][ny][nx], x fastest):
 *   fcat_image_project:     proj[r] = sum_k l_rk image[k]       (A f)
 *   fcat_image_backproject: image[k] = (accumulate ? image[k] : 0)
 *                                      + sum_r l_rk proj[r]     (A^T y)
 * with l_rk the exact length of ray r inside voxel k (Siddon's method, FP64
 * ray set-up, FP32 plane stepping as in fcat_project), so the two are each
 * other's transpose up to FP32 rounding.  proj is DEVICE float [a_end -
 * a_begin][nv][nu], image DEVICE float [nz][ny][nx].  The back-projection
 * adds with floating-point atomics: its sums are not in a fixed order
 * (results may differ in the last bits between calls).  No workspace.
 */
fcat_status fcat_image_project(const fcat_geometry_t *geometry, const fcat_grid_t *grid, const float *image,
                               int32_t a_begin, int32_t a_end, float *proj, void *stream);
fcat_status fcat_image_backproject(const fcat_geometry_t *geometry, const fcat_grid_t *grid, const float *proj,
                                   int32_t a_begin, int32_t a_end, float *image, int32_t accumulate, void *stream);

/* ---------------------------------------------------------- detector optics */
/*
 * Sec. II.B: the energy-dependent optical spread kernels, weighted by the
 * detector's energy deposition efficiency times the spectrum, give the
 * effective PSF; convolved with an idealised slit tilted by a small angle it
 * gives a line spread function, presampled to estimate the detector MTF.
 * Sec. IV.B: Richardson-Lucy deconvolution (Richardson 1972; Lucy 1974) of
 * projection images with the PSF.
 */

/* kernel (DEVICE float [k][k]) = sum_g W_g K_g / sum_g W_g, W_g = sum_{e in g} phi_e eta_e. */
fcat_status fcat_effective_psf(const fcat_spectral_t *spectral, const fcat_psf_t *psf, float *kernel, void *stream);

/*
 * Tilted slit.  Pixel (i, j) of an n_rows x n_cols image of pitch p has its
 * centre at ((j - (n_cols-1)/2) p, (i - (n_rows-1)/2) p) and holds the exact
 * fraction of its area inside the strip |x cos t + y sin t| <= width / 2
 * (t = tilt from the columns, 0 < t < 90 degrees); the image is convolved
 * with the kernel (zero outside).  Each pixel goes to bin
 * b = floor(d / h + 1/2), d = x cos t + y sin t of its centre, h = p / oversample;
 * the LSF of a bin is the mean of its pixels, and
 * mtf[f] = |sum_b LSF_b exp(-2 pi i f b h)| / |sum_b LSF_b| over the bins that
 * hold pixels (no slit-width or aperture correction).  The slit, bin and
 * MTF arithmetic is FP64; the images FP32.
 */
fcat_status fcat_slit_lsf_range(double pitch_mm, double tilt_deg, int32_t n_rows, int32_t n_cols, int32_t oversample,
                                int32_t *b_min, int32_t *n_bins);  /* HOST outputs */
size_t fcat_slit_mtf_workspace_bytes(int32_t n_rows, int32_t n_cols, int32_t n_bins);
fcat_status fcat_slit_mtf(const float *kernel, int32_t k, double pitch_mm, double width_mm, double tilt_deg,
                          int32_t n_rows, int32_t n_cols, int32_t oversample, const double *freqs, int32_t n_freq,
                          double *mtf, double *lsf, int32_t *lsf_count, void *workspace, size_t workspace_bytes,
                          void *stream);
/* freqs, mtf DEVICE double [n_freq] (cycles per mm); lsf DEVICE double [n_bins] and lsf_count
   DEVICE int32 [n_bins] (bins b_min .. b_min + n_bins - 1 of fcat_slit_lsf_range) or NULL. */

/*
 * Richardson-Lucy deconvolution of n images d (DEVICE float [n][nv][nu],
 * d >= 0) with one kernel (DEVICE float [k][k], k odd <= FCAT_MAX_PSF):
 *   u_0 = d;  u <- u (K^T (*) (d / (K (*) u))) / (K^T (*) 1)
 * with the convolution of the optical spread (zero outside the image), K^T
 * the flipped kernel, the ratio 0 where K (*) u <= 0.  out DEVICE float
 * [n][nv][nu] (not overlapping d).  n <= 65535.
 */
size_t fcat_richardson_lucy_workspace_bytes(int32_t n, int32_t nv, int32_t nu, int32_t k);
fcat_status fcat_richardson_lucy(const float *images, int32_t n, int32_t nv, int32_t nu, const float *kernel, int32_t k,
                                 int32_t iterations, float *out, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------ surrogate */
/*
 * The learned form of the primary spectral sum (see fcat_surrogate_t).  The
 * paper trains no network; it names simulated data for machine learning as
 * a use of the simulator (Sec. IV.B).  Training data are (L, Yprim) pairs of
 * rays produced by fcat_pathlengths and fcat_spectral (no scatter, I0 = 1).
 * Every product runs on the matrix cores with BF16 operands and FP32
 * accumulation (three-term hi/lo split in the forward pass, hi parts in the
 * backward pass); the FP32 parameters are the master copy.
 */

/* Number of FP32 parameters of an n_in -> 64 -> 64 -> n_out network. */
int32_t fcat_mlp_param_count(int32_t n_in, int32_t n_out);

/* Workspace needed by the fcat_mlp_* calls for up to `batch` samples per step. */
size_t fcat_mlp_workspace_bytes(const fcat_spectral_t *spectral, int64_t batch);

/* lin[g][m] = sum_{e in g} phi_e eta_e mu[m][e] / sum_{e in g} phi_e eta_e (DEVICE [G][M]). */
fcat_status fcat_mlp_linear_term(const fcat_spectral_t *spectral, float *lin, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* Network prediction of Yprim[g][r] (DEVICE [G][n]) for L (DEVICE [n][n_in]), no fallback. */
fcat_status fcat_mlp_forward(const fcat_surrogate_t *surrogate, const fcat_spectral_t *spectral,
                             const float *L, int64_t n, float *Yprim, void *workspace,
                             size_t workspace_bytes, void *stream);

/*
 * Gradient grad (DEVICE [P]) and value loss (DEVICE [1]) of the weighted
 * mean squared error, over n <= FCAT_MLP_MAX_BATCH samples and the n_out
 * groups, between out_scale[g] MLP(x)_g and the residual target
 * r_g = -ln(Yprim_g / W_g) - sum_m lin[g][m] L_m, each term weighted by
 * min(1, Yprim_g / (1e-3 sum_g Yprim_g))^2 (groups carrying less than 0.1%
 * of the ray's signal count less, as in fcat_mlp_validate).
 */
fcat_status fcat_mlp_gradients(const fcat_surrogate_t *surrogate, const fcat_spectral_t *spectral,
                               const float *L, const float *Yprim, int64_t n, float *grad, float *loss,
                               void *workspace, size_t workspace_bytes, void *stream);

/*
 * One Adam step of `train` on samples order[base .. base+count) (order:
 * DEVICE int32 [..] indices into L [n][n_in] and Yprim [G][n]; NULL means
 * base .. base+count).  count <= FCAT_MLP_MAX_BATCH.  loss (DEVICE [1] or
 * NULL) receives the batch loss before the update.  surrogate supplies
 * in_scale and lin; its params are ignored (train->params is used).
 */
fcat_status fcat_mlp_train_step(fcat_mlp_train_t *train, const fcat_surrogate_t *surrogate,
                                const fcat_spectral_t *spectral, const float *L, const float *Yprim, int64_t n,
                                const int32_t *order, int64_t base, int32_t count, float *loss,
                                void *workspace, size_t workspace_bytes, void *stream);

/* One epoch of fcat_mlp_train_step over order[0 .. n) in batches; batch_loss DEVICE [ceil(n/batch)] or NULL. */
fcat_status fcat_mlp_train_epoch(fcat_mlp_train_t *train, const fcat_surrogate_t *surrogate,
                                 const fcat_spectral_t *spectral, const float *L, const float *Yprim, int64_t n,
                                 const int32_t *order, int32_t batch, float *batch_loss, void *workspace,
                                 size_t workspace_bytes, void *stream);

/*
 * Held-out validation: for every hit ray inside the training range (see
 * fcat_surrogate_t), the largest over groups of
 * |predicted - exact| / max(exact, 1e-3 sum_g exact) is taken into its cell.
 * A group below 0.1% of the ray's signal is thus held to 1e-6 of that signal,
 * so the bound carries over to the projection sum_g K_g (*) Y_g.  cell_err
 * (DEVICE float [n_in*16] or NULL) gets the maximum per cell (inf where no
 * ray fell), cell_ok (DEVICE uint8 [n_in*16]) gets 1 where the cell holds at
 * least min_count rays and its maximum is <= threshold, cell_count (DEVICE
 * int32 [n_in*16] or NULL) the number of rays per cell.
 */
fcat_status fcat_mlp_validate(const fcat_surrogate_t *surrogate, const fcat_spectral_t *spectral,
                              const float *L, const float *Yprim, int64_t n, float threshold, int32_t min_count,
                              float *cell_err, uint8_t *cell_ok, int32_t *cell_count, void *workspace,
                              size_t workspace_bytes, void *stream);

/*
 * Set-up statistics of a training set L (DEVICE [n][n_mat]), Yprim (DEVICE
 * [G][n]) with lin from fcat_mlp_linear_term, all written to DEVICE float:
 * in_scale[m] = 1 / max(max_s L[s][m], 1e-6); out_scale[g] =
 * max(1e-3, sqrt(sum_s w r^2 / sum_s w)) with the residual target r and
 * weight w of fcat_mlp_gradients; tau_max[0] = max_s sum_m mbar_m L[s][m]
 * (mbar as in fcat_surrogate_t), the top of the cells' optical-depth range.
 * Deterministic (fixed reduction order).  Workspace: fcat_mlp_workspace_bytes.
 */
fcat_status fcat_mlp_setup(const fcat_spectral_t *spectral, const float *lin, const float *L, const float *Yprim,
                           int64_t n, float *in_scale, float *out_scale, float *tau_max, void *workspace,
                           size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------- kernel timing */

/* Kernel stages whose launches the timing facility tells apart. */
typedef enum fcat_stage FCAT_ENUM_INT {
    FCAT_STAGE_PREP = 0,   /* spectral table preparation */
    FCAT_STAGE_TRACE = 1,  /* fused traversal + contraction (or network) + spectral sum (+ scatter) */
    FCAT_STAGE_PSF = 2,    /* optical spread + group sum */
    FCAT_STAGE_MLP = 3,    /* surrogate training / inference kernels run on their own */
    FCAT_STAGE_NOISE = 4,  /* Poisson draws */
    FCAT_STAGE_PROJ = 5,   /* count scale, flood profile and log conversion */
    FCAT_STAGE_DOSE = 6,   /* dose sums over rays and bins */
    FCAT_STAGE_FILTER = 7, /* FDK cosine weight and ramp filter */
    FCAT_STAGE_BACKPROJECT = 8, /* FDK back-projection */
    FCAT_STAGE_OPTICS = 9, /* effective PSF, slit MTF, Richardson-Lucy element-wise steps */
    FCAT_STAGE_LAYOUT = 10, /* FDK: zero pads and 2 x 2 sample quads of the filtered rows */
    FCAT_STAGE_COUNT = 11
} fcat_stage;

/*
 * For benchmarks and profiling.  While enabled (process-wide), every kernel
 * that fcat_project, fcat_projections, fcat_spectral, fcat_psf and the noise
 * calls launch is bracketed by two
 * HIP events recorded on the same stream.  fcat_timing_read waits for the
 * recorded events, adds the elapsed milliseconds and launch counts per
 * stage into ms[n_stages] and launches[n_stages] (HOST arrays, either may be
 * NULL) and, if reset is non-zero, forgets them.  Events are created with
 * hipEventCreate and reused.
 */
fcat_status fcat_timing_enable(int enable);
fcat_status fcat_timing_read(double *ms, int64_t *launches, int32_t n_stages, int reset);

#ifdef __cplusplus
}
#endif

#endif /* FCAT_H */
