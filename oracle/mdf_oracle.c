/*
 * mdf_oracle.c -- plain, slow, obviously-correct FP64 implementation of the
 * multiple-distribution-function (MDF) lattice Boltzmann method with the
 * multiple-relaxation-time collision of Chai, Shi & Zhan, "Multiple-
 * distribution-function lattice Boltzmann method for convection-diffusion-
 * system based incompressible Navier-Stokes equations" (arXiv 2108.08591).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or constant
 * generator with the HIP library: every constant below is typed in again from
 * the paper.
 *
 * What it computes, in the paper's order (Remark I, eq. 3-21, which is the
 * evolution used for all of the paper's numerics):
 *   f_{i,a}(x + c_i, t + 1) = f_{i,a}(x,t) - sum_k L_{ik} [f_{k,a} - f^eq_{k,a}]
 *                             + w_i Fbar_a
 * for the d+1 sets a = 0..d (eq. 2-2: ubar_0 = rho0, ubar_a = u_a), with
 *   ubar_a = sum_i f_{i,a}                                  (eq. 2-7)
 *   P = (1/d)(sum_{a>=1} sum_i c_{i,a} f_{i,a} + cs2 R/s1 - |u|^2)  (eq. 3-15)
 *   f^eq_{i,a} = w_i [ubar_a + c_i.(ubar_a u + P E_a)/cs2]    (eq. 2-4)
 *   F_{i,a} = w_i Fbar_a, Fbar_0 = R, Fbar_a = F_a           (eq. 2-6, 2-2)
 *   L = M^{-1} S_d M                                         (eq. 4-1..4-3)
 * and the local post-processing of Section 3.3 (eq. 3-16 .. 3-19).
 *
 * With forcing = ORC_SCHEME2 the update is Scheme II (eq. 2-3c) instead:
 *   fbar_{i,a}(x + c_i, t + 1) = fbar - sum_k L_{ik} [fbar_{k,a} - f^eq_{k,a}]
 *                                + sum_k (delta_{ik} - L_{ik}/2) w_k Fbar_a
 * on the shifted populations fbar = f - F/2, with
 *   ubar_a = sum_i fbar_{i,a} + Fbar_a / 2                   (eq. 2-7a)
 * and eq. 3-15 evaluated with fbar in place of f.
 *
 * Lattice units throughout: dx = dt = c = 1.
 *
 * The paper allows a different lattice for each set a (remark after eq.
 * d3q15).  Lattice ids ORC_D2Q9_Q5 and ORC_D3Q15_Q7 run the velocity sets
 * a >= 1 on D2Q9 / D3Q15 and the set a = 0 on D2Q5 / D3Q7: every set
 * collides and streams on its own lattice (its own weights, collision matrix
 * and links); the set a = 0 occupies the first q0 entries of its row of the
 * state, the rest stay zero.
 *
 * Readings where the paper gives no formula (each is listed with its reason
 * in the design notes of the repository):
 *   - walls: the paper names an "anti-halfway bounce-back" rule for velocity
 *     Dirichlet data (Section 4) without printing it.  Read as: a link whose
 *     upstream node x - c_i lies behind a wall face or inside a solid takes
 *         f_{i,a}(x, t+1) = -f*_{ibar,a}(x, t) + 2 w_i U_{w,a}   (a >= 1)
 *         f_{i,0}(x, t+1) =  f*_{ibar,0}(x, t)                   (a = 0)
 *     where f* is the post-collision value, ibar the opposite direction and
 *     U_w the wall velocity.  Walls sit halfway between nodes.  A diagonal
 *     link (D2Q9, D3Q15) whose upstream point lies behind two or three wall
 *     faces takes the first of them in the order x, y, z.
 *   - D3Q7 transformation matrix: the paper prints none; rows e, c_x, c_y,
 *     c_z, (-6,1,1,1,1,1,1), (0,2,2,-1,-1,-1,-1), (0,0,0,1,1,-1,-1) with
 *     S_d = diag(s0, s1, s1, s1, s2, s2, s2).
 *   - initial state with a velocity gradient: f = f^eq + f^ne with
 *     f^ne_{i,a} = -(1/s1) w_i c_i . grad u_a, the inverse of eq. 3-16.
 *
 * State convention: pre-collision populations f(x, t), stored
 * array-of-structures f[node][set][dir], node = (z*ny + y)*nx + x.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_D2Q5 0
#define ORC_D3Q7 1
#define ORC_D2Q4 4
#define ORC_D3Q6 5
#define ORC_D2Q9 8
#define ORC_D3Q15 9
/* a lattice per set (the remark after eq. d3q15): the velocity sets a >= 1
 * on D2Q9 / D3Q15, the set a = 0 on D2Q5 / D3Q7 */
#define ORC_D2Q9_Q5 12
#define ORC_D3Q15_Q7 13
#define ORC_PERIODIC 0
#define ORC_WALL 1
#define ORC_PLAIN 0
#define ORC_SCHEME2 1
#define QMAX 15

typedef struct {
    int32_t lattice;        /* ORC_D2Q5, ORC_D3Q7, ORC_D2Q4, ORC_D3Q6, ORC_D2Q9 or ORC_D3Q15 */
    int32_t nx, ny, nz;     /* nz = 1 in 2D */
    double s0, s1, s2;      /* relaxation rates of S_d (eq. 4-3) */
    int32_t bc[6];          /* faces -x,+x,-y,+y,-z,+z: ORC_PERIODIC / ORC_WALL */
    double wall_u[6][3];    /* wall velocity of each face */
    double force[3];        /* uniform body force F_a, a = 1..d (eq. 2-1b) */
    double R;               /* uniform mass source R (eq. 2-1a) */
    double rho0;            /* constant density rho0 (eq. 2-2, eq. 3-17a) */
    int32_t forcing;        /* ORC_PLAIN (eq. 3-21) or ORC_SCHEME2 (eq. 2-3c) */
} orc_case;

typedef struct {
    int d, q;
    int c[QMAX][3];
    double w[QMAX];
    double cs2;
    double M[QMAX][QMAX];
    int nodd;           /* rows 1..nodd of M are odd under c -> -c and relax with s1 */
} lattice_t;

/* D2Q5 (eq. d2q5) with w_0 = 1/3 as chosen in Section 4; the transformation
 * matrix M of eq. 4-2 with c = 1. */
static void make_d2q5(lattice_t *L)
{
    static const int cx[5] = {0, 1, 0, -1, 0};
    static const int cy[5] = {0, 0, 1, 0, -1};
    static const double M[5][5] = {
        { 1,  1,  1,  1,  1},
        { 0,  1,  0, -1,  0},
        { 0,  0,  1,  0, -1},
        { 0,  1, -1,  1, -1},
        {-4,  1,  1,  1,  1},
    };
    memset(L, 0, sizeof(*L));
    L->d = 2;
    L->q = 5;
    for (int i = 0; i < 5; ++i) {
        L->c[i][0] = cx[i];
        L->c[i][1] = cy[i];
        L->c[i][2] = 0;
        L->w[i] = (i == 0) ? 1.0 / 3.0 : 1.0 / 6.0;
        for (int k = 0; k < 5; ++k) L->M[i][k] = M[i][k];
    }
    L->cs2 = 1.0 / 3.0;
    L->nodd = 2;
}

/* D3Q7 (eq. d3q7); M as read above (the paper gives none for D3Q7). */
static void make_d3q7(lattice_t *L)
{
    static const int cx[7] = {0, 1, -1, 0, 0, 0, 0};
    static const int cy[7] = {0, 0, 0, 1, -1, 0, 0};
    static const int cz[7] = {0, 0, 0, 0, 0, 1, -1};
    static const double M[7][7] = {
        { 1,  1,  1,  1,  1,  1,  1},
        { 0,  1, -1,  0,  0,  0,  0},
        { 0,  0,  0,  1, -1,  0,  0},
        { 0,  0,  0,  0,  0,  1, -1},
        {-6,  1,  1,  1,  1,  1,  1},
        { 0,  2,  2, -1, -1, -1, -1},
        { 0,  0,  0,  1,  1, -1, -1},
    };
    memset(L, 0, sizeof(*L));
    L->d = 3;
    L->q = 7;
    for (int i = 0; i < 7; ++i) {
        L->c[i][0] = cx[i];
        L->c[i][1] = cy[i];
        L->c[i][2] = cz[i];
        L->w[i] = (i == 0) ? 1.0 / 4.0 : 1.0 / 8.0;
        for (int k = 0; k < 7; ++k) L->M[i][k] = M[i][k];
    }
    L->cs2 = 1.0 / 4.0;
    L->nodd = 3;
}

/* D2Q4 (eq. d2q4), no rest population, cs^2 = 1/2.  The paper prints no M
 * for it; rows: e, c_x, c_y and the remaining even moment c_x^2 - c_y^2,
 * with S_d = diag(s0, s1, s1, s2). */
static void make_d2q4(lattice_t *L)
{
    static const int cx[4] = {1, 0, -1, 0};
    static const int cy[4] = {0, 1, 0, -1};
    static const double M[4][4] = {
        { 1,  1,  1,  1},
        { 1,  0, -1,  0},
        { 0,  1,  0, -1},
        { 1, -1,  1, -1},
    };
    memset(L, 0, sizeof(*L));
    L->d = 2;
    L->q = 4;
    for (int i = 0; i < 4; ++i) {
        L->c[i][0] = cx[i];
        L->c[i][1] = cy[i];
        L->c[i][2] = 0;
        L->w[i] = 1.0 / 4.0;
        for (int k = 0; k < 4; ++k) L->M[i][k] = M[i][k];
    }
    L->cs2 = 1.0 / 2.0;
    L->nodd = 2;
}

/* D3Q6 (eq. d3q6), no rest population, cs^2 = 1/3.  No M in the paper;
 * rows: e, c_x, c_y, c_z, 2c_x^2 - c_y^2 - c_z^2 and c_y^2 - c_z^2, with
 * S_d = diag(s0, s1, s1, s1, s2, s2). */
static void make_d3q6(lattice_t *L)
{
    static const int cx[6] = {1, -1, 0, 0, 0, 0};
    static const int cy[6] = {0, 0, 1, -1, 0, 0};
    static const int cz[6] = {0, 0, 0, 0, 1, -1};
    static const double M[6][6] = {
        { 1,  1,  1,  1,  1,  1},
        { 1, -1,  0,  0,  0,  0},
        { 0,  0,  1, -1,  0,  0},
        { 0,  0,  0,  0,  1, -1},
        { 2,  2, -1, -1, -1, -1},
        { 0,  0,  1,  1, -1, -1},
    };
    memset(L, 0, sizeof(*L));
    L->d = 3;
    L->q = 6;
    for (int i = 0; i < 6; ++i) {
        L->c[i][0] = cx[i];
        L->c[i][1] = cy[i];
        L->c[i][2] = cz[i];
        L->w[i] = 1.0 / 6.0;
        for (int k = 0; k < 6; ++k) L->M[i][k] = M[i][k];
    }
    L->cs2 = 1.0 / 3.0;
    L->nodd = 3;
}

/* Fill L from velocities and weights; M from a list of row functions. */
static void fill_lattice(lattice_t *L, int d, int q, const int (*c)[3], const double *w, double cs2,
                         int nodd, const double (*M)[QMAX])
{
    memset(L, 0, sizeof(*L));
    L->d = d;
    L->q = q;
    L->cs2 = cs2;
    L->nodd = nodd;
    for (int i = 0; i < q; ++i) {
        for (int b = 0; b < 3; ++b) L->c[i][b] = c[i][b];
        L->w[i] = w[i];
        for (int r = 0; r < q; ++r) L->M[r][i] = M[r][i];
    }
}

/* D2Q9 (eq. d2q9), cs^2 = 1/3.  The paper prints no M for it.  Rows, in
 * the usual moment basis: e; the odd moments c_x, c_y and the energy fluxes
 * (3|c|^2 - 5) c_x, (3|c|^2 - 5) c_y; the even moments 3|c|^2 - 4,
 * (9|c|^4 - 21|c|^2 + 8)/2, c_x^2 - c_y^2 and c_x c_y.  S_d keeps the
 * structure of eq. 4-3: s0 on e, s1 on every odd row, s2 on every even one. */
static void make_d2q9(lattice_t *L)
{
    static const int c[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    double w[9], M[QMAX][QMAX];
    memset(M, 0, sizeof M);
    for (int i = 0; i < 9; ++i) {
        const int cx = c[i][0], cy = c[i][1], c2 = cx * cx + cy * cy;
        w[i] = c2 == 0 ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        M[0][i] = 1;
        M[1][i] = cx;
        M[2][i] = cy;
        M[3][i] = (3 * c2 - 5) * cx;
        M[4][i] = (3 * c2 - 5) * cy;
        M[5][i] = 3 * c2 - 4;
        M[6][i] = (9.0 * c2 * c2 - 21.0 * c2 + 8.0) / 2.0;
        M[7][i] = cx * cx - cy * cy;
        M[8][i] = cx * cy;
    }
    fill_lattice(L, 2, 9, c, w, 1.0 / 3.0, 4, (const double (*)[QMAX])M);
}

/* D3Q15 (eq. d3q15), cs^2 = 1/3, velocities in the column order printed.
 * No M in the paper.  Rows: e; odd: c_x, c_y, c_z, (5|c|^2 - 13) c_b for
 * each b, and c_x c_y c_z; even: |c|^2 - 2, (15|c|^4 - 55|c|^2 + 32)/2,
 * 3c_x^2 - |c|^2, c_y^2 - c_z^2, c_x c_y, c_y c_z, c_z c_x.  s1 on every odd
 * row, s2 on every even one. */
static void make_d3q15(lattice_t *L)
{
    static const int c[15][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
                                 {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}, {-1, -1, 1}, {-1, 1, -1},
                                 {1, -1, -1}, {-1, -1, -1}};
    double w[15], M[QMAX][QMAX];
    memset(M, 0, sizeof M);
    for (int i = 0; i < 15; ++i) {
        const int cx = c[i][0], cy = c[i][1], cz = c[i][2], c2 = cx * cx + cy * cy + cz * cz;
        w[i] = c2 == 0 ? 2.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 72.0);
        M[0][i] = 1;
        M[1][i] = cx;
        M[2][i] = cy;
        M[3][i] = cz;
        M[4][i] = (5 * c2 - 13) * cx;
        M[5][i] = (5 * c2 - 13) * cy;
        M[6][i] = (5 * c2 - 13) * cz;
        M[7][i] = cx * cy * cz;
        M[8][i] = c2 - 2;
        M[9][i] = (15.0 * c2 * c2 - 55.0 * c2 + 32.0) / 2.0;
        M[10][i] = 3 * cx * cx - c2;
        M[11][i] = cy * cy - cz * cz;
        M[12][i] = cx * cy;
        M[13][i] = cy * cz;
        M[14][i] = cz * cx;
    }
    fill_lattice(L, 3, 15, c, w, 1.0 / 3.0, 7, (const double (*)[QMAX])M);
}

static int make_lattice(int lattice, lattice_t *L)
{
    if (lattice == ORC_D2Q9_Q5) { make_d2q9(L); return 0; }
    if (lattice == ORC_D3Q15_Q7) { make_d3q15(L); return 0; }
    if (lattice == ORC_D2Q5) { make_d2q5(L); return 0; }
    if (lattice == ORC_D3Q7) { make_d3q7(L); return 0; }
    if (lattice == ORC_D2Q4) { make_d2q4(L); return 0; }
    if (lattice == ORC_D3Q6) { make_d3q6(L); return 0; }
    if (lattice == ORC_D2Q9) { make_d2q9(L); return 0; }
    if (lattice == ORC_D3Q15) { make_d3q15(L); return 0; }
    return -1;
}

/* The lattice of the set a = 0: its own for a mixed lattice id, else the
 * lattice of every set. */
static int make_set0_lattice(int lattice, lattice_t *L0)
{
    if (lattice == ORC_D2Q9_Q5) { make_d2q5(L0); return 0; }
    if (lattice == ORC_D3Q15_Q7) { make_d3q7(L0); return 0; }
    return make_lattice(lattice, L0);
}

/* opposite direction: the j with c_j = -c_i */
static int opposite(const lattice_t *L, int i)
{
    for (int j = 0; j < L->q; ++j)
        if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
            L->c[j][2] == -L->c[i][2])
            return j;
    return -1;
}

/* Gauss-Jordan inverse with partial pivoting of an n x n matrix. */
static int invert(int n, const double A[QMAX][QMAX], double Ainv[QMAX][QMAX])
{
    double a[QMAX][2 * QMAX];
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < 2 * n; ++k)
            a[r][k] = (k < n) ? A[r][k] : (k - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int k = 0; k < 2 * n; ++k) {
                double t = a[col][k]; a[col][k] = a[piv][k]; a[piv][k] = t;
            }
        double p = a[col][col];
        for (int k = 0; k < 2 * n; ++k) a[col][k] /= p;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double m = a[r][col];
            if (m != 0.0)
                for (int k = 0; k < 2 * n; ++k) a[r][k] -= m * a[col][k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < n; ++k) Ainv[r][k] = a[r][n + k];
    return 0;
}

/* Collision matrix L = M^{-1} S_d M (eq. 4-1), S_d = diag(s0, s1.., s2..)
 * (eq. 4-3): s0 on the conserved row, s1 on the d first-order rows, s2 on the
 * remaining rows. */
static int collision_matrix(const lattice_t *L, double s0, double s1, double s2,
                            double Lam[QMAX][QMAX])
{
    double Minv[QMAX][QMAX], S[QMAX];
    int q = L->q, d = L->d;
    if (invert(q, L->M, Minv) != 0) return -1;
    (void)d;
    for (int r = 0; r < q; ++r) S[r] = (r == 0) ? s0 : (r <= L->nodd ? s1 : s2);
    for (int i = 0; i < q; ++i)
        for (int k = 0; k < q; ++k) {
            double acc = 0.0;
            for (int r = 0; r < q; ++r) acc += Minv[i][r] * S[r] * L->M[r][k];
            Lam[i][k] = acc;
        }
    return 0;
}

static double default_s2(double s1)
{
    /* s2 = 8(2 - s1)/(8 - s1), the choice used for all runs of Section 4 */
    return 8.0 * (2.0 - s1) / (8.0 - s1);
}

static double relax_s2(const orc_case *cs)
{
    return cs->s2 > 0.0 ? cs->s2 : default_s2(cs->s1);
}

/* ---------------------------------------------------------------- moments */

typedef struct {
    double ubar[4];     /* ubar_a, a = 0..d (eq. 2-7) */
    double u[3];        /* u_b = ubar_{b+1} */
    double J[4][3];     /* J_{a,b} = sum_i c_{i,b} f_{i,a} */
    double P;           /* eq. 3-15 */
} moments_t;

/* Fbar_a at node n, a = 0..d (eq. 2-2): Fbar_0 = R, Fbar_a = F_a plus the
 * per-node force field (component-major, d*N values) when one is given. */
static void node_source(const orc_case *cs, int d, const double *force_field, long N, long n,
                        double *Fbar)
{
    Fbar[0] = cs->R;
    for (int a = 1; a <= d; ++a) {
        Fbar[a] = cs->force[a - 1];
        if (force_field) Fbar[a] += force_field[(a - 1) * N + n];
    }
}

/* Moments of the stored populations fn of one node.  Fbar is used only by
 * Scheme II, whose ubar is eq. 2-7a. */
static void node_moments(const lattice_t *L, const lattice_t *L0, const orc_case *cs,
                         const double *fn /* [set][dir] */, const double *Fbar, moments_t *m)
{
    int d = L->d, q = L->q;
    memset(m, 0, sizeof(*m));
    for (int a = 0; a <= d; ++a) {
        const lattice_t *La = (a == 0) ? L0 : L;      /* the lattice of set a */
        double s = 0.0;
        for (int i = 0; i < La->q; ++i) s += fn[a * q + i];
        if (cs->forcing == ORC_SCHEME2) s += 0.5 * Fbar[a];      /* eq. 2-7a */
        m->ubar[a] = s;
        for (int b = 0; b < d; ++b) {
            double j = 0.0;
            for (int i = 0; i < La->q; ++i) j += La->c[i][b] * fn[a * q + i];
            m->J[a][b] = j;
        }
    }
    for (int b = 0; b < d; ++b) m->u[b] = m->ubar[b + 1];
    double trJ = 0.0, u2 = 0.0;
    for (int a = 1; a <= d; ++a) trJ += m->J[a][a - 1];
    for (int b = 0; b < d; ++b) u2 += m->u[b] * m->u[b];
    m->P = (trJ + L->cs2 * cs->R / cs->s1 - u2) / d;
}

/* f^eq_{i,a} = w_i [ubar_a + c_i . (ubar_a u + P E_a) / cs2]   (eq. 2-4);
 * E_0 = 0 and E_a is the a-th unit vector. */
static void equilibrium(const lattice_t *L, int a, double ubar_a, const double *u,
                        double P, double *feq)
{
    for (int i = 0; i < L->q; ++i) {
        double cflux = 0.0;
        for (int b = 0; b < L->d; ++b) {
            double flux_b = ubar_a * u[b] + ((a >= 1 && b == a - 1) ? P : 0.0);
            cflux += L->c[i][b] * flux_b;
        }
        feq[i] = L->w[i] * (ubar_a + cflux / L->cs2);
    }
}

static long nodes_of(const orc_case *cs)
{
    return (long)cs->nx * cs->ny * cs->nz;
}

static int check_case(const orc_case *cs, lattice_t *L, lattice_t *L0)
{
    if (make_lattice(cs->lattice, L) != 0) return -1;
    if (make_set0_lattice(cs->lattice, L0) != 0) return -1;
    if (cs->nx < 1 || cs->ny < 1 || cs->nz < 1) return -1;
    if (L->d == 2 && cs->nz != 1) return -1;
    if (!(cs->s1 > 0.0 && cs->s1 < 2.0)) return -1;
    if (cs->forcing != ORC_PLAIN && cs->forcing != ORC_SCHEME2) return -1;
    return 0;
}

/* ------------------------------------------------------------- public API */

/* Lattice tables: c (q x 3, row-major), w (q), cs2, M (q x q). */
int orc_lattice_info(int lattice, int *d, int *q, int *c, double *w, double *cs2,
                     double *M)
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    *d = L.d;
    *q = L.q;
    *cs2 = L.cs2;
    for (int i = 0; i < L.q; ++i) {
        w[i] = L.w[i];
        for (int b = 0; b < 3; ++b) c[i * 3 + b] = L.c[i][b];
        for (int k = 0; k < L.q; ++k) M[i * L.q + k] = L.M[i][k];
    }
    return 0;
}

/* Lattice id of the set a = 0 for a lattice id (the id itself unless the
 * set a = 0 has a lattice of its own), or -1. */
int orc_set0_lattice(int lattice)
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    if (lattice == ORC_D2Q9_Q5) return ORC_D2Q5;
    if (lattice == ORC_D3Q15_Q7) return ORC_D3Q7;
    return lattice;
}

/* Collision matrix L = M^{-1} S_d M, row-major q x q.  s2 <= 0 selects the
 * default s2 = 8(2 - s1)/(8 - s1). */
int orc_collision_matrix(int lattice, double s0, double s1, double s2, double *out)
{
    lattice_t L;
    double Lam[QMAX][QMAX];
    if (make_lattice(lattice, &L) != 0) return -1;
    if (s2 <= 0.0) s2 = default_s2(s1);
    if (collision_matrix(&L, s0, s1, s2, Lam) != 0) return -1;
    for (int i = 0; i < L.q; ++i)
        for (int k = 0; k < L.q; ++k) out[i * L.q + k] = Lam[i][k];
    return 0;
}

/* Initial populations f(x, 0) from macroscopic fields.
 *   P:    N values;  u: d*N values, component-major (u[b*N + node]);
 *   grad: d*d*N values or NULL, grad[((a-1)*d + b)*N + node] = d u_a / d x_b.
 * f = f^eq(rho0, u, P) (eq. 2-4) plus, when grad is given, the
 * non-equilibrium part f^ne_{i,a} = -(1/s1) w_i c_i . grad u_a (inverse of
 * eq. 3-16; the set a = 0 carries the constant rho0 and gets none).
 * Scheme II stores fbar = f - F/2, F_{i,a} = w_i Fbar_a (force_field as in
 * orc_collide), so that eq. 2-7a returns the given ubar.
 * solid may be NULL; solid nodes are set to zero. */
int orc_init(const orc_case *cs, const uint8_t *solid, const double *force_field,
             const double *P, const double *u, const double *grad, double *f)
{
    lattice_t L, L0;
    if (check_case(cs, &L, &L0) != 0) return -1;
    long N = nodes_of(cs);
    int d = L.d, q = L.q, ns = d + 1;
    for (long n = 0; n < N; ++n) {
        double *fn = f + n * ns * q;
        for (int k = 0; k < ns * q; ++k) fn[k] = 0.0;
        if (solid && solid[n]) continue;
        double un[3] = {0, 0, 0};
        for (int b = 0; b < d; ++b) un[b] = u[b * N + n];
        for (int a = 0; a <= d; ++a) {
            const lattice_t *La = (a == 0) ? &L0 : &L;
            double ubar_a = (a == 0) ? cs->rho0 : un[a - 1];
            double feq[QMAX];
            equilibrium(La, a, ubar_a, un, P[n], feq);
            for (int i = 0; i < La->q; ++i) {
                double fne = 0.0;
                if (grad && a >= 1) {
                    double cg = 0.0;
                    for (int b = 0; b < d; ++b)
                        cg += La->c[i][b] * grad[((a - 1) * d + b) * N + n];
                    fne = -(1.0 / cs->s1) * La->w[i] * cg;
                }
                fn[a * q + i] = feq[i] + fne;
            }
        }
        if (cs->forcing == ORC_SCHEME2) {
            double Fbar[4];
            node_source(cs, d, force_field, N, n, Fbar);
            for (int a = 0; a <= d; ++a) {
                const lattice_t *La = (a == 0) ? &L0 : &L;
                for (int i = 0; i < La->q; ++i) fn[a * q + i] -= 0.5 * La->w[i] * Fbar[a];
            }
        }
    }
    return 0;
}

/* Collision at every fluid node (right-hand side of eq. 3-21):
 *   fpost_{i,a} = f_{i,a} - sum_k L_{ik} (f_{k,a} - f^eq_{k,a}) + w_i Fbar_a,
 * or under Scheme II (right-hand side of eq. 2-3c, f standing for fbar):
 *   fpost_{i,a} = f_{i,a} - sum_k L_{ik} (f_{k,a} - f^eq_{k,a})
 *                 + sum_k (delta_{ik} - L_{ik}/2) w_k Fbar_a.
 * force_field: d*N values (component-major) added to the uniform force, or
 * NULL. */
int orc_collide(const orc_case *cs, const uint8_t *solid, const double *force_field,
                const double *f, double *fpost)
{
    lattice_t L, L0;
    double Lam[QMAX][QMAX], Lam0[QMAX][QMAX];
    if (check_case(cs, &L, &L0) != 0) return -1;
    if (collision_matrix(&L, cs->s0, cs->s1, relax_s2(cs), Lam) != 0) return -1;
    if (collision_matrix(&L0, cs->s0, cs->s1, relax_s2(cs), Lam0) != 0) return -1;
    long N = nodes_of(cs);
    int d = L.d, q = L.q, ns = d + 1;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        const double *fn = f + n * ns * q;
        double *fo = fpost + n * ns * q;
        for (int k = 0; k < ns * q; ++k) fo[k] = 0.0;
        if (solid && solid[n]) continue;
        double Fbar[4];
        node_source(cs, d, force_field, N, n, Fbar);
        moments_t m;
        node_moments(&L, &L0, cs, fn, Fbar, &m);
        for (int a = 0; a <= d; ++a) {
            /* each set collides on its own lattice (the same for every set
             * unless the set a = 0 has one of its own) */
            const lattice_t *La = (a == 0) ? &L0 : &L;
            double (*LamA)[QMAX] = (a == 0) ? Lam0 : Lam;
            const int qa = La->q;
            double feq[QMAX], fne[QMAX];
            equilibrium(La, a, m.ubar[a], m.u, m.P, feq);
            for (int i = 0; i < qa; ++i) fne[i] = fn[a * q + i] - feq[i];
            for (int i = 0; i < qa; ++i) {
                double coll = 0.0;
                for (int k = 0; k < qa; ++k) coll += LamA[i][k] * fne[k];
                double src = La->w[i] * Fbar[a];
                if (cs->forcing == ORC_SCHEME2) {
                    /* (I - L/2) applied to F_{k,a} = w_k Fbar_a */
                    double lf = 0.0;
                    for (int k = 0; k < qa; ++k) lf += LamA[i][k] * La->w[k] * Fbar[a];
                    src -= 0.5 * lf;
                }
                fo[a * q + i] = fn[a * q + i] - coll + src;
            }
        }
    }
    return 0;
}

/* Which wall face (0..5) the upstream point x - c_i falls behind, or -1 if
 * it is inside the box.  *wrapped receives the periodic image. */
static int upstream(const orc_case *cs, const lattice_t *L, int x, int y, int z,
                    int i, int *sx, int *sy, int *sz)
{
    int p[3] = {x - L->c[i][0], y - L->c[i][1], z - L->c[i][2]};
    int n[3] = {cs->nx, cs->ny, cs->nz};
    for (int b = 0; b < 3; ++b) {
        if (p[b] < 0) {
            if (cs->bc[2 * b] == ORC_WALL) return 2 * b;
            p[b] += n[b];
        } else if (p[b] >= n[b]) {
            if (cs->bc[2 * b + 1] == ORC_WALL) return 2 * b + 1;
            p[b] -= n[b];
        }
    }
    *sx = p[0];
    *sy = p[1];
    *sz = p[2];
    return -1;
}

/* Streaming (left-hand side of eq. 3-21): f_{i,a}(x, t+1) = fpost_{i,a}(x - c_i, t),
 * periodic faces wrap; links from behind a wall face or from a solid node use
 * the halfway anti-bounce-back reading stated in the file header. */
int orc_stream(const orc_case *cs, const uint8_t *solid, const double *fpost, double *f)
{
    lattice_t L, L0;
    if (check_case(cs, &L, &L0) != 0) return -1;
    int d = L.d, q = L.q, ns = d + 1;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < cs->nz; ++z)
        for (int y = 0; y < cs->ny; ++y)
            for (int x = 0; x < cs->nx; ++x) {
                long n = ((long)z * cs->ny + y) * cs->nx + x;
                double *fn = f + n * ns * q;
                for (int k = 0; k < ns * q; ++k) fn[k] = 0.0;
                if (solid && solid[n]) continue;
                const double *own = fpost + n * ns * q;
                for (int a = 0; a < ns; ++a) {
                    const lattice_t *La = (a == 0) ? &L0 : &L;     /* the lattice of set a */
                    for (int i = 0; i < La->q; ++i) {
                        int sx = 0, sy = 0, sz = 0;
                        int face = upstream(cs, La, x, y, z, i, &sx, &sy, &sz);
                        const double *Uw = NULL;
                        static const double zero[3] = {0, 0, 0};
                        if (face >= 0) {
                            Uw = cs->wall_u[face];
                        } else {
                            long sn = ((long)sz * cs->ny + sy) * cs->nx + sx;
                            if (solid && solid[sn]) {
                                Uw = zero;
                            } else {
                                fn[a * q + i] = fpost[sn * ns * q + a * q + i];
                                continue;
                            }
                        }
                        /* link crosses a wall: bounce back (a = 0) or
                         * anti-bounce-back with the wall velocity (a >= 1) */
                        const int j = opposite(La, i);
                        if (a == 0) fn[i] = own[j];
                        else fn[a * q + i] = -own[a * q + j] + 2.0 * La->w[i] * Uw[a - 1];
                    }
                }
            }
    return 0;
}

/* Number of field channels written by orc_fields. */
int orc_num_fields(int lattice)
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    int d = L.d;
    int nsym = d * (d + 1) / 2;
    int nvort = (d == 2) ? 1 : 3;
    return (d + 1) + 1 + d * d + 1 + nsym + nsym + nvort;
}

/* Macroscopic and derived fields at time t from pre-collision f(x, t),
 * channel-major out[ch*N + node], channels in this order:
 *   ubar_0..ubar_d               eq. 2-7
 *   P                            eq. 3-15
 *   grad u: d*d, (a-1)*d + b     eq. 3-16  (d u_a / d x_b)
 *   div u                        eq. 3-16a
 *   S: symmetric, (xx,xy,yy) in 2D, (xx,xy,xz,yy,yz,zz) in 3D   eq. 3-17
 *   sigma: same order            eq. 3-17a
 *   vorticity: omega (2D) or (omega_x, omega_y, omega_z) (3D), from the
 *   antisymmetric tensor Omega (eq. 3-18) through eq. 3-19.
 * Under Scheme II, f holds fbar; the non-equilibrium part is taken of the
 * unshifted f = fbar + F/2 (force_field as in orc_collide).
 * Solid nodes get zeros. */
int orc_fields(const orc_case *cs, const uint8_t *solid, const double *force_field,
               const double *f, double *out)
{
    lattice_t L, L0;
    if (check_case(cs, &L, &L0) != 0) return -1;
    long N = nodes_of(cs);
    int d = L.d, q = L.q, ns = d + 1;
    int nch = orc_num_fields(cs->lattice);
    double s1 = cs->s1, cs2 = L.cs2;
    for (long n = 0; n < N; ++n) {
        if (solid && solid[n]) {
            for (int ch = 0; ch < nch; ++ch) out[ch * N + n] = 0.0;
            continue;
        }
        const double *fn = f + n * ns * q;
        double Fbar[4];
        node_source(cs, d, force_field, N, n, Fbar);
        moments_t m;
        node_moments(&L, &L0, cs, fn, Fbar, &m);
        /* first moment of the non-equilibrium part, mne[a][b] =
         * sum_i c_{i,b} f^ne_{i,a}, a = 1..d */
        double mne[4][3];
        for (int a = 1; a <= d; ++a) {
            double feq[QMAX];
            equilibrium(&L, a, m.ubar[a], m.u, m.P, feq);
            for (int b = 0; b < d; ++b) {
                double acc = 0.0;
                for (int i = 0; i < q; ++i) {
                    double fi = fn[a * q + i];
                    if (cs->forcing == ORC_SCHEME2) fi += 0.5 * L.w[i] * Fbar[a];
                    acc += L.c[i][b] * (fi - feq[i]);
                }
                mne[a][b] = acc;
            }
        }
        int ch = 0;
        for (int a = 0; a <= d; ++a) out[(ch++) * N + n] = m.ubar[a];
        out[(ch++) * N + n] = m.P;
        /* eq. 3-16: grad_b u_a = -(s1 / (cs2 dt)) sum_i c_{i,b} f^ne_{i,a} */
        double G[3][3];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                G[a][b] = -(s1 / cs2) * mne[a + 1][b];
                out[(ch++) * N + n] = G[a][b];
            }
        /* eq. 3-16a */
        double dv = 0.0;
        for (int a = 1; a <= d; ++a) dv += mne[a][a - 1];
        out[(ch++) * N + n] = -(s1 / cs2) * dv;
        /* eq. 3-17 */
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b)
                out[(ch++) * N + n] =
                    -(s1 / (2.0 * cs2)) * (mne[a + 1][b] + mne[b + 1][a]);
        /* eq. 3-17a */
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b)
                out[(ch++) * N + n] =
                    -cs->rho0 * (1.0 - s1 / 2.0) * (mne[a + 1][b] + mne[b + 1][a]);
        /* eq. 3-18, Omega_{ab} = -(s1/(2 cs2)) sum_i (c_{i,b} f^ne_{i,a} - c_{i,a} f^ne_{i,b}) */
        double Om[3][3];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
                Om[a][b] = -(s1 / (2.0 * cs2)) * (mne[a + 1][b] - mne[b + 1][a]);
        /* eq. 3-19, Omega_{ab} = -1/2 eps_{abg} omega_g, so
         * omega_g = -sum_{a,b} eps_{abg} Omega_{ab}.  In 2D the flow lies in
         * the (x, y) plane and only omega_z survives. */
        if (d == 2) {
            double om = 0.0;
            /* eps_{12 3} = +1, eps_{21 3} = -1 */
            om = -(Om[0][1] - Om[1][0]);
            out[(ch++) * N + n] = om;
        } else {
            for (int g = 0; g < 3; ++g) {
                double om = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        int e = 0;
                        /* Levi-Civita symbol */
                        if (a != b && b != g && a != g)
                            e = ((a == 0 && b == 1 && g == 2) || (a == 1 && b == 2 && g == 0) ||
                                 (a == 2 && b == 0 && g == 1)) ? 1 : -1;
                        om -= e * Om[a][b];
                    }
                out[(ch++) * N + n] = om;
            }
        }
    }
    return 0;
}

/* One full time step: collide then stream.  f holds f(., t) on entry and
 * f(., t+1) on return; tmp is N*(d+1)*q doubles of scratch. */
int orc_step(const orc_case *cs, const uint8_t *solid, const double *force_field,
             double *f, double *tmp)
{
    if (orc_collide(cs, solid, force_field, f, tmp) != 0) return -1;
    return orc_stream(cs, solid, tmp, f);
}

/* nsteps time steps. */
int orc_run(const orc_case *cs, const uint8_t *solid, const double *force_field,
            double *f, double *tmp, long nsteps)
{
    for (long s = 0; s < nsteps; ++s)
        if (orc_step(cs, solid, force_field, f, tmp) != 0) return -1;
    return 0;
}

/* ------------------------------------------------ 16-bit deviation storage
 *
 * Not in the paper: the library can store each post-collision population as
 * a 16-bit floating-point deviation from the rest state,
 *     stored = (f - f_rest) / u_ref,   f = f_rest + u_ref * stored,
 * f_rest_{i,0} = w_i rho0 and f_rest_{i,a>=1} = 0, and collide in binary32.
 * The oracle keeps its FP64 arithmetic and takes the one rounding decision
 * of the format in the precision the library takes it in: f, f_rest and
 * 1/u_ref are rounded to binary32, the deviation is formed and scaled in
 * binary32, and the result is rounded to the nearest value of the 16-bit
 * format, ties to even.  The decoded value is then formed in FP64.
 *   ORC_BINARY16: IEEE 754 binary16, 11-bit significand, exponents -14..15
 *                 (subnormals below 2^-14), largest finite 65504.
 *   ORC_BFLOAT16: bfloat16, 8-bit significand, the exponent range of
 *                 binary32 (subnormals below 2^-126). */
#define ORC_BINARY16 2
#define ORC_BFLOAT16 3

/* Nearest value of the 16-bit format to the binary32 value x, ties to even:
 * x is a multiple of the spacing of its binade, q = 2^(e - p + 1) with e the
 * exponent of x (at least emin) and p the significand bits, so x / q is
 * exact in FP64 and rint() (round to nearest even, the default mode) picks
 * the neighbour.  Beyond the largest finite value the result is infinite. */
static double round16(int fmt, float x)
{
    const int p = (fmt == ORC_BINARY16) ? 11 : 8;
    const int emin = (fmt == ORC_BINARY16) ? -14 : -126;
    const int emax = (fmt == ORC_BINARY16) ? 15 : 127;
    double v = (double)x;
    if (isnan(v) || isinf(v) || v == 0.0) return v;
    int e = ilogb(v);
    if (e < emin) e = emin;
    double q = ldexp(1.0, e - p + 1);
    double y = rint(v / q) * q;
    /* largest finite value (2 - 2^(1-p)) 2^emax; a result above it overflowed */
    double big = ldexp(2.0 - ldexp(1.0, 1 - p), emax);
    if (fabs(y) > big) return copysign(INFINITY, v);
    return y;
}

/* out[k] = the 16-bit value nearest to in[k] (binary32), as a double. */
int orc_round16(int fmt, const float *in, double *out, long n)
{
    if (fmt != ORC_BINARY16 && fmt != ORC_BFLOAT16) return -1;
    for (long k = 0; k < n; ++k) out[k] = round16(fmt, in[k]);
    return 0;
}

/* Replace every population of the fluid nodes of f ([node][set][dir]) by
 * its round trip through the 16-bit deviation storage described above. */
int orc_store16(const orc_case *cs, const uint8_t *solid, int fmt, double u_ref, double *f)
{
    lattice_t L, L0;
    if (check_case(cs, &L, &L0) != 0) return -1;
    if ((fmt != ORC_BINARY16 && fmt != ORC_BFLOAT16) || !(u_ref > 0.0)) return -1;
    long N = nodes_of(cs);
    int d = L.d, q = L.q, ns = d + 1;
    const float inv32 = (float)(1.0 / u_ref);
    for (long n = 0; n < N; ++n) {
        if (solid && solid[n]) continue;
        double *fn = f + n * ns * q;
        for (int a = 0; a < ns; ++a)
            for (int i = 0; i < ((a == 0) ? L0.q : q); ++i) {
                const double rest = (a == 0) ? L0.w[i] * cs->rho0 : 0.0;
                const float v32 = (float)fn[a * q + i];
                const float r32 = (float)rest;
                const float dev32 = (v32 - r32) * inv32;        /* binary32 operations */
                fn[a * q + i] = rest + u_ref * round16(fmt, dev32);
            }
    }
    return 0;
}

/* nsteps steps with the 16-bit storage: collide, store the post-collision
 * populations through the format, stream. */
int orc_run16(const orc_case *cs, const uint8_t *solid, const double *force_field, int fmt, double u_ref,
              double *f, double *tmp, long nsteps)
{
    for (long s = 0; s < nsteps; ++s) {
        if (orc_collide(cs, solid, force_field, f, tmp) != 0) return -1;
        if (orc_store16(cs, solid, fmt, u_ref, tmp) != 0) return -1;
        if (orc_stream(cs, solid, tmp, f) != 0) return -1;
    }
    return 0;
}

/* Global sums over fluid nodes of pre-collision f(., t):
 *   out[a] = sum_x ubar_a for a = 0..d,
 *   out[d+1] = sum_x sum_{a>=1} J_{a,a}.
 * force_field as in orc_collide (it enters ubar under Scheme II). */
int orc_invariants(const orc_case *cs, const uint8_t *solid, const double *force_field,
                   const double *f, double *out)
{
    lattice_t L, L0;
    if (check_case(cs, &L, &L0) != 0) return -1;
    long N = nodes_of(cs);
    int d = L.d, q = L.q, ns = d + 1;
    for (int k = 0; k < d + 2; ++k) out[k] = 0.0;
    for (long n = 0; n < N; ++n) {
        if (solid && solid[n]) continue;
        double Fbar[4];
        node_source(cs, d, force_field, N, n, Fbar);
        moments_t m;
        node_moments(&L, &L0, cs, f + n * ns * q, Fbar, &m);
        for (int a = 0; a <= d; ++a) out[a] += m.ubar[a];
        for (int a = 1; a <= d; ++a) out[d + 1] += m.J[a][a - 1];
    }
    return 0;
}
