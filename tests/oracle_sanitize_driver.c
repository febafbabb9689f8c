/*
 * Host sanitizer run of the FP64 oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py, it drives the oracle's entry points over a
 * tiny random phantom, including rays that miss, rays parallel to an axis,
 * rays in a voxel plane and a bad label, and checks the results that have a
 * closed form.  Exit status 0 and "ok" on success.
 */
#include "../oracle/fcat_oracle.c"

#include <stdio.h>

static uint64_t rng = 88172645463325252ull;
static double urand(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(void)
{
    enum { NX = 6, NY = 5, NZ = 4, M = 3, E = 7, G = 2, NU = 9, NV = 4, A = 3, K = 5 };
    int8_t lab[NZ * NY * NX];
    for (int i = 0; i < NZ * NY * NX; ++i) lab[i] = (int8_t)(urand() * M);
    orc_volume v = {NX, NY, NZ, 1.0, 1.25, 0.75, 0.3, -0.2, 0.1, lab};
    orc_geometry g = {40.0, 60.0, NU, NV, 1.5, 1.2, 0.25, -0.1, A, NULL};

    /* Siddon against brute force, and the total length against the chord */
    double L[M], Lb[M];
    for (int r = 0; r < 40; ++r) {
        double s[3], d[3];
        for (int ax = 0; ax < 3; ++ax) {
            s[ax] = (urand() - 0.5) * 30.0;
            d[ax] = (urand() - 0.5) * 30.0;
        }
        if (r % 5 == 0) d[2] = s[2];            /* parallel to the xy plane */
        if (r % 7 == 0) { s[0] = d[0] = 0.3; }  /* in a voxel plane (x = cx) */
        CHECK(orc_siddon(s, d, &v, M, L) == ORC_OK);
        CHECK(orc_bruteforce(s, d, &v, M, 200000, Lb) == ORC_OK);
        for (int m = 0; m < M; ++m) CHECK(fabs(L[m] - Lb[m]) < 2e-3);
    }
    /* a ray that misses the grid */
    double s0[3] = {100.0, 100.0, 100.0}, d0[3] = {120.0, 90.0, 100.0};
    CHECK(orc_siddon(s0, d0, &v, M, L) == ORC_OK);
    for (int m = 0; m < M; ++m) CHECK(L[m] == 0.0);

    /* the full projector with flood, scatter, per-bin scatter scale, groups and PSF */
    double mu[M * E], phi[E], eta[E], sb[E], flood[NV * NU], S[A * NV * NU], Kr[G * K * K];
    int32_t grp[E], idx[A];
    for (int i = 0; i < M * E; ++i) mu[i] = 0.01 + 0.2 * urand();
    for (int e = 0; e < E; ++e) {
        phi[e] = urand();
        eta[e] = 0.5 + 0.5 * urand();
        sb[e] = 0.5 + urand();
        grp[e] = e < 3 ? 0 : 1;
    }
    for (int i = 0; i < NV * NU; ++i) flood[i] = 0.8 + 0.4 * urand();
    for (int i = 0; i < A * NV * NU; ++i) S[i] = 0.1 * urand();
    for (int i = 0; i < G * K * K; ++i) Kr[i] = urand();
    for (int a = 0; a < A; ++a) idx[a] = a;
    double out[A * NV * NU], Y[A * G * NV * NU];
    CHECK(orc_project(&g, &v, M, E, G, mu, phi, eta, grp, flood, S, sb, Kr, K, idx, A, out, Y, 1) == ORC_OK);
    for (int i = 0; i < A * NV * NU; ++i) CHECK(isfinite(out[i]) && out[i] > 0.0);
    /* without the spread, out is the group sum */
    double out2[A * NV * NU];
    CHECK(orc_project(&g, &v, M, E, G, mu, phi, eta, grp, NULL, NULL, NULL, NULL, 0, idx, A, out2, NULL, 1) == ORC_OK);
    for (int i = 0; i < A * NV * NU; ++i) CHECK(isfinite(out2[i]));

    /* a label outside 0 .. M-1 is reported, not read past the tables: a ray
       along z through the centre of voxel 7 = (ix 1, iy 1, iz 0) */
    lab[7] = (int8_t)M;
    const double x0 = 0.3 - NX * 1.0 / 2, y0 = -0.2 - NY * 1.25 / 2;
    double bs[3] = {x0 + 1.5 * 1.0, y0 + 1.5 * 1.25, -5.0}, bd[3] = {bs[0], bs[1], 5.0};
    CHECK(orc_siddon(bs, bd, &v, M, L) == ORC_BAD_LABEL);
    CHECK(orc_bruteforce(bs, bd, &v, M, 1000, Lb) == ORC_BAD_LABEL);
    printf("ok\n");
    return 0;
}
