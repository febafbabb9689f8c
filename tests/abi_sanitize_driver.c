/*
 * Host sanitizer run of the C ABI's host code (test infrastructure): built
 * with AddressSanitizer and UndefinedBehaviorSanitizer on the host side of
 * every library source by tests/test_abi_sanitizers.py, it drives the
 * argument validation, the group-map parsing, the workspace layouts and the
 * chunk arithmetic of every entry point with valid and invalid descriptors.
 * Nothing here reaches the GPU: every call either only sizes a workspace or
 * is rejected before its first HIP call.  Exit status 0 and "ok" on success.
 */
#include "../include/fcat.h"

#include <stdio.h>
#include <string.h>

#define CHECK(c)                                                                    \
    do {                                                                            \
        if (!(c)) {                                                                 \
            fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #c,     \
                    fcat_last_error());                                             \
            return 1;                                                               \
        }                                                                           \
    } while (0)

#define DEV(x) ((void *)(uintptr_t)(x))

int main(void)
{
    fcat_geometry_t geo = {1000.0, 1520.0, 1024, 64, 0.392, 0.392, 0.0, 0.0, 360, NULL};
    fcat_phantom_t ph = {256, 256, 200, 0.15625, 0.15625, 0.15625, 0.0, 0.0, 0.0, (const int8_t *)DEV(0x1000)};
    fcat_spectral_t sp = {8, 200, 8, DEV(0x2000), DEV(0x3000), DEV(0x4000), NULL, NULL};
    fcat_psf_t psf = {15, DEV(0x5000)};
    fcat_scatter_t sc = {DEV(0x6000), NULL};
    const fcat_mode modes[3] = {FCAT_MODE_PLAIN, FCAT_MODE_SPLIT_BF16, FCAT_MODE_SURROGATE};

    /* status strings, including unknown codes */
    for (int s = -2; s < 10; ++s) CHECK(fcat_status_string((fcat_status)s) != NULL);
    CHECK(fcat_version() == FCAT_VERSION);

    /* workspace sizes over modes, chunks and the optional stages */
    for (int m = 0; m < 3; ++m)
        for (int chunk = 0; chunk < 400; chunk += 37) {
            size_t a = fcat_project_workspace_bytes(&geo, &ph, &sp, &sc, &psf, modes[m], chunk);
            size_t b = fcat_project_workspace_bytes(&geo, &ph, &sp, NULL, NULL, modes[m], chunk);
            size_t c = fcat_projections_workspace_bytes(&geo, &ph, &sp, &sc, &psf, modes[m], chunk);
            CHECK(a > 0 && b > 0 && c >= a && a % 256 == 0);
        }
    CHECK(fcat_dose_workspace_bytes(&geo, &ph, &sp, 0) > 0 && fcat_dose_workspace_bytes(&geo, &ph, &sp, 7) > 0);
    CHECK(fcat_fdk_workspace_bytes(&geo, 0) > 0 && fcat_fdk_workspace_bytes(&geo, 5) > 0);
    CHECK(fcat_pathlengths_workspace_bytes(&ph) > 0 && fcat_spectral_workspace_bytes(&sp) > 0);
    CHECK(fcat_flood_workspace_bytes(&sp, 64, 1024) > 0 && fcat_mlp_workspace_bytes(&sp, 4096) > 0);
    CHECK(fcat_richardson_lucy_workspace_bytes(360, 64, 1024, 15) > 0);
    CHECK(fcat_fdk_backproject_workspace_bytes(360) > 0 && fcat_mlp_param_count(10, 8) == 5384);

    /* explicit group maps: valid, a gap, a decrease, out of range */
    int32_t gob[200];
    for (int e = 0; e < 200; ++e) gob[e] = e * 8 / 200;
    sp.group_of_bin = gob;
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &sp, &sc, &psf, FCAT_MODE_SPLIT_BF16, 0) > 0);
    gob[100] = 7;
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &sp, &sc, &psf, FCAT_MODE_PLAIN, 0) == 0);
    gob[100] = 4;
    gob[199] = 8;
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &sp, &sc, &psf, FCAT_MODE_PLAIN, 0) == 0);
    gob[199] = 7;
    gob[50] = 0;
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &sp, &sc, &psf, FCAT_MODE_PLAIN, 0) == 0);
    sp.group_of_bin = NULL;

    /* descriptor limits: sizes, distances, materials, energies, groups, k */
    fcat_geometry_t g2 = geo;
    g2.sdd_mm = 900.0;
    CHECK(fcat_project_workspace_bytes(&g2, &ph, &sp, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    g2 = geo;
    g2.nu = 0;
    CHECK(fcat_project_workspace_bytes(&g2, &ph, &sp, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    g2 = geo;
    g2.nu = 1 << 20;
    g2.nv = 1 << 20;
    CHECK(fcat_project_workspace_bytes(&g2, &ph, &sp, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    fcat_phantom_t p2 = ph;
    p2.nx = 1024;
    p2.ny = 2048;
    p2.nz = 1024;
    CHECK(fcat_project_workspace_bytes(&geo, &p2, &sp, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    p2.nx = 2047;                                /* < 2^31 voxels, 2^31 once rounded up to bricks */
    p2.ny = 1024;
    CHECK(fcat_project_workspace_bytes(&geo, &p2, &sp, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    p2.nx = 256;                                 /* 2^30 voxels: accepted */
    p2.ny = 2048;
    p2.nz = 2048;
    CHECK(fcat_project_workspace_bytes(&geo, &p2, &sp, NULL, NULL, FCAT_MODE_PLAIN, 0) > 0);
    p2 = ph;
    p2.nx = 2147483647;
    p2.ny = 1;
    p2.nz = 1;
    CHECK(fcat_project_workspace_bytes(&geo, &p2, &sp, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    fcat_spectral_t s2 = sp;
    s2.n_mat = FCAT_MAX_MATERIALS + 1;
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &s2, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    s2 = sp;
    s2.n_groups = 201;
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &s2, NULL, NULL, FCAT_MODE_PLAIN, 0) == 0);
    s2 = sp;
    s2.n_energy = FCAT_MAX_ENERGIES;
    s2.n_groups = FCAT_MAX_GROUPS;
    s2.n_mat = FCAT_MAX_MATERIALS;
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &s2, &sc, &psf, FCAT_MODE_SPLIT_BF16, 1) > 0);
    fcat_psf_t k2 = {14, DEV(0x5000)};
    CHECK(fcat_project_workspace_bytes(&geo, &ph, &sp, NULL, &k2, FCAT_MODE_PLAIN, 0) == 0);

    /* entry points rejected before any launch */
    void *ws = DEV(0x100000);   /* an aligned device address, never dereferenced on the host */
    CHECK(fcat_project(NULL, &ph, &sp, NULL, NULL, FCAT_MODE_PLAIN, NULL, DEV(0x7000), ws, 64, NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_project(&geo, &ph, &sp, NULL, NULL, FCAT_MODE_PLAIN, NULL, DEV(0x7000), ws, 64, NULL) ==
          FCAT_E_WORKSPACE);
    CHECK(fcat_project(&geo, &ph, &sp, NULL, NULL, FCAT_MODE_SURROGATE, NULL, DEV(0x7000), ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_project(&geo, &ph, &sp, NULL, NULL, (fcat_mode)7, NULL, DEV(0x7000), ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    fcat_noise_t nz = {-1.0, 5, 0.0f};
    CHECK(fcat_projections(&geo, &ph, &sp, NULL, NULL, FCAT_MODE_PLAIN, NULL, &nz, DEV(0x7000), ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_project_status(NULL, 0, NULL) == FCAT_E_WORKSPACE);
    CHECK(fcat_pathlengths(&geo, &ph, 8, 6, 5, DEV(0x7000), ws, 1 << 30, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_walk_stats(&geo, &ph, 0, 1, NULL, ws, 1 << 30, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_spectral(DEV(0x7000), -1, &sp, NULL, NULL, NULL, FCAT_MODE_PLAIN, DEV(0x8000), ws, 1 << 20, NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_spectral_static(DEV(0x7000), 10, &sp, NULL, NULL, NULL, FCAT_MODE_SURROGATE, DEV(0x8000), NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_spectral_static(DEV(0x7000), 0, &sp, NULL, NULL, NULL, FCAT_MODE_PLAIN, NULL, NULL) == FCAT_OK);
    CHECK(fcat_psf(DEV(0x7000), 3, 8, 64, 1024, NULL, DEV(0x8000), NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_check_inputs(&geo, &ph, &sp, NULL, NULL, ws, 8, NULL) == FCAT_E_WORKSPACE);
    CHECK(fcat_count_scale(&sp, 0.0, DEV(0x7000), NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_poisson(DEV(0x7000), -1, 8, 100, DEV(0x8000), 1, 0, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_log_projection(DEV(0x7000), NULL, 3, 100, 0.0f, DEV(0x7000), NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_dose(&geo, &ph, &sp, DEV(0x7000), DEV(0x7000), -1.0, 0, 1, DEV(0x8000), NULL, ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    g2 = geo;
    g2.nu = 8192;
    CHECK(fcat_fdk_filter(&g2, DEV(0x7000), 3, DEV(0x8000000), NULL) == FCAT_E_UNSUPPORTED);
    fcat_grid_t grid = {64, 64, 8, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0};
    fcat_grid_t bad_grid = {64, 64, 0, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0};
    CHECK(fcat_fdk(&geo, DEV(0x7000), &bad_grid, DEV(0x8000), ws, 1 << 30, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_image_project(&geo, &grid, DEV(0x7000), 3, 2, DEV(0x8000), NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_image_backproject(&geo, &grid, NULL, 0, 1, DEV(0x8000), 0, NULL) == FCAT_E_INVALID_ARG);
    int32_t bmin = 0, nbins = 0;
    CHECK(fcat_slit_lsf_range(0.392, 2.5, 256, 64, 10, &bmin, &nbins) == FCAT_OK && nbins > 0);
    CHECK(fcat_slit_lsf_range(0.392, 95.0, 256, 64, 10, &bmin, &nbins) == FCAT_E_INVALID_ARG);
    CHECK(fcat_slit_mtf(DEV(0x7000), 15, 0.392, 0.3, 2.5, 256, 64, 0, DEV(0x8000), 10, DEV(0x9000), NULL, NULL, ws,
                        1 << 30, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_richardson_lucy(DEV(0x7000), 1, 8, 8, DEV(0x8000), 14, 3, DEV(0x9000), ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_effective_psf(&sp, NULL, DEV(0x7000), NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_mlp_linear_term(NULL, DEV(0x7000), ws, 1 << 20, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_mlp_forward(NULL, &sp, DEV(0x7000), 10, DEV(0x8000), ws, 1 << 20, NULL) == FCAT_E_INVALID_ARG);
    fcat_mlp_train_t tr = {DEV(0x7000), DEV(0x7100), DEV(0x7200), 0, 1e-3f, 0.9f, 0.999f, 1e-8f};
    CHECK(fcat_mlp_train_step(&tr, NULL, &sp, DEV(0x7000), DEV(0x7000), 10, NULL, 0, 4, NULL, ws, 1 << 20, NULL) ==
          FCAT_E_INVALID_ARG);
    fcat_surrogate_t su = {7, 8, DEV(0xa000), DEV(0xa100), DEV(0xa200), DEV(0xa300), (const uint8_t *)DEV(0xa400),
                           0.0f, 8.0f, NULL};                    /* n_in != n_mat */
    CHECK(fcat_project(&geo, &ph, &sp, NULL, NULL, FCAT_MODE_SURROGATE, &su, DEV(0x7000), ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    su.n_in = 8;
    su.cell_lo = 8.0f;                                           /* empty optical-depth range */
    CHECK(fcat_project(&geo, &ph, &sp, NULL, NULL, FCAT_MODE_SURROGATE, &su, DEV(0x7000), ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_fdk_backproject(&geo, DEV(0x7000), 5, 3, &grid, DEV(0x8000), 0, ws, 1 << 30, NULL) ==
          FCAT_E_INVALID_ARG);
    CHECK(fcat_flood_profile(&sp, &psf, 0, 1024, DEV(0x7000), ws, 1 << 30, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_mlp_validate(&su, &sp, DEV(0x7000), DEV(0x7100), 10, -1.0f, 1, DEV(0x8000), (uint8_t *)DEV(0x8100),
                            (int32_t *)DEV(0x8200), ws, 1 << 30, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_mlp_setup(&sp, DEV(0x7000), DEV(0x7100), DEV(0x7200), -5, DEV(0x8000), DEV(0x8100), DEV(0x8200), ws,
                         1 << 30, NULL) == FCAT_E_INVALID_ARG);
    CHECK(fcat_timing_read(NULL, NULL, -1, 0) == FCAT_E_INVALID_ARG);
    CHECK(strlen(fcat_last_error()) > 0);
    printf("ok\n");
    return 0;
}
