/*
 * oracle_sanitize.c -- drives every entry point of the FP64 oracle over small
 * grids of every lattice, with walls, moving walls, obstacles, a force field,
 * a mass source and both forcing schemes, plus the 16-bit storage emulation
 * and the refused arguments.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers_cpu.py; every buffer is
 * allocated at exactly the size the oracle's interface states, so a read or
 * write past it, an uninitialised index or an integer overflow stops the run.
 * Test infrastructure only.
 */
#include "mdf_oracle.c"

#include <stdio.h>

static int fails = 0;

#define CHECK(cond)                                                            \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__);  \
            ++fails;                                                           \
        }                                                                      \
    } while (0)

static double *alloc(long n)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (long k = 0; k < n; ++k) p[k] = 0.0;
    return p;
}

static int all_finite(const double *p, long n)
{
    for (long k = 0; k < n; ++k)
        if (!isfinite(p[k])) return 0;
    return 1;
}

/* One case: init with a gradient, three plain steps, fields, invariants,
 * three 16-bit steps in each format. */
static void run_case(int lattice, int nx, int ny, int nz, int walls, int mask, int scheme2, int field)
{
    int d, q, c[QMAX * 3];
    double w[QMAX], cs2, M[QMAX * QMAX];
    CHECK(orc_lattice_info(lattice, &d, &q, c, w, &cs2, M) == 0);
    orc_case cs;
    memset(&cs, 0, sizeof cs);
    cs.lattice = lattice;
    cs.nx = nx;
    cs.ny = ny;
    cs.nz = nz;
    cs.s0 = 1.0;
    cs.s1 = 1.3;
    cs.s2 = walls ? 0.0 : 1.1;
    cs.rho0 = 1.0;
    cs.R = walls ? 0.0 : 1e-4;
    cs.forcing = scheme2 ? ORC_SCHEME2 : ORC_PLAIN;
    for (int b = 0; b < d; ++b) cs.force[b] = 1e-5 * (b + 1);
    if (walls) {
        for (int f = 2; f < 2 * d; ++f) cs.bc[f] = ORC_WALL;
        cs.wall_u[3][0] = 0.05;
        if (d == 3) cs.wall_u[4][1] = 0.01;
    }
    const long N = (long)nx * ny * nz;
    const long nf = N * (d + 1) * q;
    uint8_t *solid = NULL;
    if (mask) {
        solid = (uint8_t *)calloc((size_t)N, 1);
        for (long n = N / 3; n < N / 3 + nx / 2; ++n) solid[n] = 1;
    }
    double *ff = field ? alloc(d * N) : NULL;
    if (ff)
        for (long k = 0; k < d * N; ++k) ff[k] = 1e-6 * (double)(k % 7);
    double *P = alloc(N), *u = alloc(d * N), *grad = alloc(d * d * N);
    for (long n = 0; n < N; ++n) {
        P[n] = 1e-3 * sin(0.3 * (double)n);
        for (int b = 0; b < d; ++b) u[b * N + n] = 0.02 * cos(0.2 * (double)n + b);
        for (int k = 0; k < d * d; ++k) grad[k * N + n] = 1e-3 * sin(0.1 * (double)(n + k));
    }
    double *f = alloc(nf), *tmp = alloc(nf), *f16 = alloc(nf);
    CHECK(orc_init(&cs, solid, ff, P, u, grad, f) == 0);
    memcpy(f16, f, sizeof(double) * (size_t)nf);
    CHECK(orc_run(&cs, solid, ff, f, tmp, 3) == 0);
    CHECK(all_finite(f, nf));
    const int nch = orc_num_fields(lattice);
    CHECK(nch > 0);
    double *out = alloc((long)nch * N), inv[5];
    CHECK(orc_fields(&cs, solid, ff, f, out) == 0);
    CHECK(all_finite(out, (long)nch * N));
    CHECK(orc_invariants(&cs, solid, ff, f, inv) == 0);
    CHECK(all_finite(inv, d + 2));
    for (int fmt = ORC_BINARY16; fmt <= ORC_BFLOAT16; ++fmt) {
        memcpy(tmp, f16, sizeof(double) * (size_t)nf);
        double *g = alloc(nf);
        memcpy(g, f16, sizeof(double) * (size_t)nf);
        CHECK(orc_run16(&cs, solid, ff, fmt, 0.05, g, tmp, 3) == 0);
        CHECK(all_finite(g, nf));
        free(g);
    }
    free(out);
    free(f16);
    free(tmp);
    free(f);
    free(grad);
    free(u);
    free(P);
    free(ff);
    free(solid);
}

int main(void)
{
    static const int lat2[] = {ORC_D2Q5, ORC_D2Q4, ORC_D2Q9, ORC_D2Q9_Q5};
    static const int lat3[] = {ORC_D3Q7, ORC_D3Q6, ORC_D3Q15, ORC_D3Q15_Q7};
    int cases = 0;
    for (int k = 0; k < 4; ++k) {
        for (int v = 0; v < 4; ++v) {
            run_case(lat2[k], 9, 7, 1, v & 1, v >> 1, v == 3, v == 2);
            run_case(lat3[k], 6, 5, 4, v & 1, v >> 1, v == 3, v == 2);
            cases += 2;
        }
        double Lm[QMAX * QMAX];
        CHECK(orc_collision_matrix(lat2[k], 1.0, 1.2, 0.0, Lm) == 0);
        CHECK(orc_collision_matrix(lat3[k], 1.0, 1.2, 1.5, Lm) == 0);
        CHECK(orc_set0_lattice(lat2[k]) >= 0 && orc_set0_lattice(lat3[k]) >= 0);
    }
    /* refused arguments */
    int d, q, c[QMAX * 3];
    double w[QMAX], cs2, M[QMAX * QMAX], one = 0.0;
    CHECK(orc_lattice_info(99, &d, &q, c, w, &cs2, M) == -1);
    CHECK(orc_set0_lattice(-1) == -1);
    CHECK(orc_collision_matrix(99, 1.0, 1.2, 0.0, M) == -1);
    orc_case bad;
    memset(&bad, 0, sizeof bad);
    bad.lattice = ORC_D2Q5;
    bad.nx = 4;
    bad.ny = 4;
    bad.nz = 2;              /* 2D with nz != 1 */
    bad.s1 = 1.0;
    CHECK(orc_run(&bad, NULL, NULL, &one, &one, 1) == -1);
    bad.nz = 1;
    bad.s1 = 2.5;            /* outside (0, 2) */
    CHECK(orc_fields(&bad, NULL, NULL, &one, &one) == -1);
    bad.s1 = 1.0;
    bad.forcing = 7;
    CHECK(orc_invariants(&bad, NULL, NULL, &one, &one) == -1);
    float x = 1.0f;
    CHECK(orc_round16(9, &x, &one, 1) == -1);
    CHECK(orc_round16(ORC_BINARY16, &x, &one, 1) == 0 && one == 1.0);
    printf("oracle sanitizer run: %d cases, %d failed checks\n", cases, fails);
    return fails != 0;
}
