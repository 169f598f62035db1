/*
 * FP64 CPU oracle for the explicit EDF-based MesoFD / MMFD time step
 * (Shi, Du & Chai, "Equilibrium-distribution-function based mesoscopic
 * finite-difference methods for partial differential equations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it is used by the test suite, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no code, header, table or
 * constant generator with the GPU library.
 *
 * It is deliberately plain: whole-grid loops in IEEE binary64, no blocking,
 * no fusion, periodic wrap by modular indexing.  Build with
 *   gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * so that every a*b+c below is a rounded multiply followed by a rounded add.
 * OpenMP only splits the outer node loop; every node's arithmetic is the same
 * with any thread count, so results are bitwise independent of threads.
 *
 * Notation (lattice units, c = dx/dt = 1, c_s^2 = d0):
 *   e_j, w_j      lattice velocities and weights (Appendix A; D1Q3 from the
 *                 pattern w_j = d0/2, w_0 = 1 - 2 sum w_j of Eq. (LMMFD-4))
 *   a_k, ah_k     scheme coefficients at time levels t and t-dt, k = -1,0,+1
 *                 (three-level notation of Eq. (3layer-1)); a two-level
 *                 explicit scheme is the case ah = 0.
 *   g_j(A,B,C)    quadratic EDF of Eqs. (3-3)/(3-4):
 *                 w_j [ A + e_j.B/d0 + sum_a C_aa (e_ja^2-d0)/(d0(1-d0))
 *                       + sum_{a!=b} C_ab e_ja e_jb /(2 d0^2) ]
 *   g+_p, g-_p    even / odd parts of g over an opposite pair p=(j, jbar),
 *                 Eq. (2-5): g+ = w (A + Q:C), g- = w e.B/d0 (the split of
 *                 Eq. (TforMMFD-2) applied to the general EDF).
 *
 * Every floating-point expression is evaluated left to right in the order
 * written; sums over lattice directions run in Appendix-A order, over k in
 * the order -1, 0, +1, level t before level t-dt.
 *
 * Parity status: every function below is pinned by a CPU test (Fourier
 * symbol, FTCS identity, textbook LBGK equilibrium, EDF moment identities,
 * exact rational brute force, conservation, convergence to analytic
 * solutions; the source term by its Fourier symbol, the literal form,
 * conservation and second-order convergence on Example 1).  The paper's
 * Table 1/2/3 error values are NOT reproduced and are not used as pins.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_D1Q3 = 1, ORC_D2Q5 = 2, ORC_D2Q9 = 3, ORC_D3Q19 = 4, ORC_D2Q5II = 5, ORC_D3Q7 = 6,
       ORC_D3Q9 = 7, ORC_D3Q27 = 8 };
enum { ORC_LCDE = 0, ORC_BURGERS = 1, ORC_NSE = 2, ORC_WAVE = 3 };

#define ORC_MAXQ 27
#define ORC_MAXP 13

typedef struct {
    int32_t lattice;      /* ORC_D1Q3 ...                                    */
    int32_t eq;           /* ORC_LCDE / ORC_BURGERS / ORC_NSE / ORC_WAVE     */
    int32_t levels;       /* 2: two-level explicit, 3: three-level explicit  */
    int32_t lambda_bar;   /* LCDE: 1 adds u u to C (Eq. TforMMFD-0)          */
    int32_t he_luo;       /* NSE: C = j j / rho0 (Remark 4)                  */
    int32_t nthreads;     /* 0: OpenMP default                               */
    int32_t theta_iters;  /* Jacobi sweeps per theta step                    */
    int32_t bc;           /* 0 periodic, 1 Dirichlet edges (2D, scalar)      */
    int64_t n[3];         /* nodes along x, y, z (x fastest)                 */
    double d0, dx, dt;
    double u[3];          /* LCDE advection velocity (physical)              */
    double K[9];          /* LCDE diffusion tensor (physical, row major)     */
    double beta;          /* NCDE: D = phi I scaled by beta (Eq. NCDEfeq)    */
    double rho0;          /* NSE: reference density; the state holds rho-rho0*/
    double a[3], ah[3];   /* k = -1, 0, +1 at level t and t-dt               */
    double ab[3], abh[3]; /* momentum parameter set of Eq. (2-4)             */
    double theta;         /* weight of the old level, Eq. (GCN)              */
    /* Dirichlet edges: the nodes with x or y = 0 or n-1 of the level a step
     * writes hold bG[i] * bscale (bscale = exp(lambda t) of that level,
     * evaluated by the caller); bG has one value per node (edges read) */
    double bscale;
    const double *bG;
    /* multiple-set parameters, Eq. (2-2-1b) / (2-1b) (scalar equations):
     * multiset = 1 takes the Delta^2 (even) terms from ae/aeh and the
     * Delta^1 (odd) terms from ao/aoh; a/ah keep the base terms */
    int32_t multiset;
    int32_t pad2_;
    double ae[3], aeh[3], ao[3], aoh[3];
    /* rectangular lattice of Appendix A (linear CDE): rect = 1 takes the
     * spacing dxv[a] and d0v[a] = c_s,a^2 / c_a^2 per axis in place of dx
     * and d0 (axes beyond the dimension ignored) */
    int32_t rect;
    int32_t pad3_;
    double d0v[3], dxv[3];
    /* linear CDE: -A10 / A22 of the scheme when > 0 (schemes beyond the
     * three-level one, Eq. (4-2-00a) moments of their own coefficients);
     * 0: from a / ah */
    double ratio;
} orc_params;

typedef struct {
    int dim, b, npair;
    int e[ORC_MAXQ][3];
    double w[ORC_MAXQ];
    int opp[ORC_MAXQ];
    int pair[ORC_MAXP];   /* representative direction of each opposite pair */
} orc_lattice;

/* ---------------------------------------------------------------- lattices */

static void set_e(orc_lattice *L, int j, int x, int y, int z)
{
    L->e[j][0] = x; L->e[j][1] = y; L->e[j][2] = z;
}

/* Appendix A with d0_alpha = d0 on every axis (square / cubic grids). */
/* Weights of Appendix A with d0_a = dv[a] per axis (equal values: the
 * square / cubic lattice); rD2Q5II and rD3Q9 take one d0 (dv[0]). */
static int build_lattice_v(int lattice, const double *dv, orc_lattice *L)
{
    const double d0 = dv[0], dx = dv[0], dy = dv[1], dz = dv[2];
    memset(L, 0, sizeof(*L));
    if (lattice == ORC_D1Q3) {
        L->dim = 1; L->b = 3;
        set_e(L, 0, 0, 0, 0); set_e(L, 1, 1, 0, 0); set_e(L, 2, -1, 0, 0);
        L->w[0] = 1.0 - dx;
        L->w[1] = dx / 2.0;
        L->w[2] = dx / 2.0;
    } else if (lattice == ORC_D2Q5) {
        L->dim = 2; L->b = 5;
        set_e(L, 0, 0, 0, 0); set_e(L, 1, 1, 0, 0); set_e(L, 2, 0, 1, 0);
        set_e(L, 3, -1, 0, 0); set_e(L, 4, 0, -1, 0);
        L->w[0] = 1.0 - dx - dy;
        L->w[1] = dx / 2.0; L->w[3] = L->w[1];
        L->w[2] = dy / 2.0; L->w[4] = L->w[2];
    } else if (lattice == ORC_D2Q9) {
        L->dim = 2; L->b = 9;
        set_e(L, 0, 0, 0, 0); set_e(L, 1, 1, 0, 0); set_e(L, 2, 0, 1, 0);
        set_e(L, 3, -1, 0, 0); set_e(L, 4, 0, -1, 0); set_e(L, 5, 1, 1, 0);
        set_e(L, 6, -1, 1, 0); set_e(L, 7, -1, -1, 0); set_e(L, 8, 1, -1, 0);
        L->w[0] = (1.0 - dx) * (1.0 - dy);
        L->w[1] = dx * (1.0 - dy) / 2.0; L->w[3] = L->w[1];
        L->w[2] = (1.0 - dx) * dy / 2.0; L->w[4] = L->w[2];
        L->w[5] = dx * dy / 4.0;
        L->w[6] = L->w[5]; L->w[7] = L->w[5]; L->w[8] = L->w[5];
    } else if (lattice == ORC_D3Q19 || lattice == ORC_D3Q27) {
        /* The xz-edge block of the printed tables repeats two velocities; the
         * edge sets here follow the xy pattern (+,+),(-,+),(-,-),(+,-).
         * rD3Q27 adds the eight corners in the printed order. */
        static const int E[27][3] = {
            {0,0,0}, {1,0,0}, {0,1,0}, {0,0,1}, {-1,0,0}, {0,-1,0}, {0,0,-1},
            {1,1,0}, {-1,1,0}, {-1,-1,0}, {1,-1,0},
            {1,0,1}, {-1,0,1}, {-1,0,-1}, {1,0,-1},
            {0,1,1}, {0,-1,1}, {0,-1,-1}, {0,1,-1},
            {1,1,1}, {1,1,-1}, {1,-1,1}, {-1,1,1},
            {-1,-1,-1}, {-1,-1,1}, {-1,1,-1}, {1,-1,-1}};
        const int b = lattice == ORC_D3Q19 ? 19 : 27;
        L->dim = 3; L->b = b;
        for (int j = 0; j < b; ++j) set_e(L, j, E[j][0], E[j][1], E[j][2]);
        if (lattice == ORC_D3Q19) {
            L->w[0] = 1.0 - dx - dy - dz + dx * dy + dx * dz + dy * dz;
            L->w[1] = dx * (1.0 - dy - dz) / 2.0; L->w[4] = L->w[1];
            L->w[2] = dy * (1.0 - dx - dz) / 2.0; L->w[5] = L->w[2];
            L->w[3] = dz * (1.0 - dx - dy) / 2.0; L->w[6] = L->w[3];
            for (int j = 7; j <= 10; ++j) L->w[j] = dx * dy / 4.0;
            for (int j = 11; j <= 14; ++j) L->w[j] = dx * dz / 4.0;
            for (int j = 15; j <= 18; ++j) L->w[j] = dy * dz / 4.0;
        } else {
            L->w[0] = (1.0 - dx) * (1.0 - dy) * (1.0 - dz);
            L->w[1] = dx * (1.0 - dy) * (1.0 - dz) / 2.0; L->w[4] = L->w[1];
            L->w[2] = dy * (1.0 - dx) * (1.0 - dz) / 2.0; L->w[5] = L->w[2];
            L->w[3] = dz * (1.0 - dx) * (1.0 - dy) / 2.0; L->w[6] = L->w[3];
            for (int j = 7; j <= 10; ++j) L->w[j] = dx * dy * (1.0 - dz) / 4.0;
            for (int j = 11; j <= 14; ++j) L->w[j] = dx * dz * (1.0 - dy) / 4.0;
            for (int j = 15; j <= 18; ++j) L->w[j] = dy * dz * (1.0 - dx) / 4.0;
            for (int j = 19; j <= 26; ++j) L->w[j] = dx * dy * dz / 8.0;
        }
    } else if (lattice == ORC_D2Q5II) {
        /* the rest velocity and the four diagonals, weights d0 / 4 */
        if (dy != d0) return -1;
        L->dim = 2; L->b = 5;
        set_e(L, 0, 0, 0, 0); set_e(L, 1, 1, 1, 0); set_e(L, 2, -1, 1, 0);
        set_e(L, 3, -1, -1, 0); set_e(L, 4, 1, -1, 0);
        L->w[0] = 1.0 - d0;
        for (int j = 1; j <= 4; ++j) L->w[j] = d0 / 4.0;
    } else if (lattice == ORC_D3Q7) {
        /* the rest velocity and the six axis directions, weights d0_a / 2 */
        L->dim = 3; L->b = 7;
        set_e(L, 0, 0, 0, 0); set_e(L, 1, 1, 0, 0); set_e(L, 2, 0, 1, 0);
        set_e(L, 3, 0, 0, 1); set_e(L, 4, -1, 0, 0); set_e(L, 5, 0, -1, 0);
        set_e(L, 6, 0, 0, -1);
        L->w[0] = 1.0 - dx - dy - dz;
        L->w[1] = dx / 2.0; L->w[4] = L->w[1];
        L->w[2] = dy / 2.0; L->w[5] = L->w[2];
        L->w[3] = dz / 2.0; L->w[6] = L->w[3];
    } else if (lattice == ORC_D3Q9) {
        /* the rest velocity and the eight cube corners, weights d0 / 8 */
        if (dy != d0 || dz != d0) return -1;
        static const int E[9][3] = {
            {0,0,0}, {1,1,1}, {1,1,-1}, {1,-1,1}, {-1,1,1},
            {-1,-1,-1}, {-1,-1,1}, {-1,1,-1}, {1,-1,-1}};
        L->dim = 3; L->b = 9;
        for (int j = 0; j < 9; ++j) set_e(L, j, E[j][0], E[j][1], E[j][2]);
        L->w[0] = 1.0 - d0;
        for (int j = 1; j <= 8; ++j) L->w[j] = d0 / 8.0;
    } else {
        return -1;
    }
    /* opposite directions and pair representatives (first of each pair) */
    for (int j = 0; j < L->b; ++j) {
        L->opp[j] = -1;
        for (int i = 0; i < L->b; ++i)
            if (L->e[i][0] == -L->e[j][0] && L->e[i][1] == -L->e[j][1] &&
                L->e[i][2] == -L->e[j][2])
                L->opp[j] = i;
    }
    for (int j = 1; j < L->b; ++j)
        if (L->opp[j] > j) L->pair[L->npair++] = j;
    return 0;
}

static int build_lattice(int lattice, double d0, orc_lattice *L)
{
    const double dv[3] = {d0, d0, d0};
    return build_lattice_v(lattice, dv, L);
}

/* ------------------------------------------------- derived constant tables */

typedef struct {
    orc_lattice L;
    int dim;
    int64_t n[3], N;
    double inv_d0;
    int rect;                 /* per-axis d0 (rectangular lattice)           */
    double inv_d0v[3];        /* 1 / d0_a                                    */
    double qd[ORC_MAXQ][3];   /* (e_a^2 - d0) / (d0 (1 - d0))                */
    double qo[ORC_MAXQ][3];   /* e_a e_b / d0^2 for (a,b) = (0,1),(0,2),(1,2)*/
    double w1[ORC_MAXQ];      /* w_j / d0                                    */
    /* scheme */
    double A0, Ah0, Ab0, Abh0;
    double ap, am, ahp, ahm;      /* a+ = a_1 + a_-1, a- = a_1 - a_-1       */
    double abp, abm, abhp, abhm;  /* same for the momentum set              */
    /* LCDE */
    double uh[3], kh[9], Ch[9];
    double ubar[ORC_MAXQ];        /* full  g_j(1, uh, Ch)                    */
    double ubp[ORC_MAXP], ubm[ORC_MAXP];   /* even / odd parts per pair      */
    double Cp[ORC_MAXP], Cm[ORC_MAXP], Chp[ORC_MAXP], Chm[ORC_MAXP];
    /* Burgers */
    double bh, cbeta;
    int beta_one;
    /* NSE */
    double rho0, rinv0;
    int he_luo;
} orc_ctx;

static const int OFF_A[3] = {0, 0, 1};
static const int OFF_B[3] = {1, 2, 2};

/* sum_a qd_ja C_aa + sum_{a<b} qo_jab C_ab, accumulated left to right */
static double quad_term(const orc_ctx *c, int j, const double *C)
{
    int d = c->dim;
    double t = c->qd[j][0] * C[0];
    for (int a = 1; a < d; ++a) t = t + c->qd[j][a] * C[a * 3 + a];
    int no = d == 1 ? 0 : (d == 2 ? 1 : 3);
    for (int o = 0; o < no; ++o) {
        if (c->qo[j][o] != 0.0) t = t + c->qo[j][o] * C[OFF_A[o] * 3 + OFF_B[o]];
    }
    return t;
}

/* e_j . B with e in {-1,0,1}: signed accumulation from zero */
static double edot(const orc_ctx *c, int j, const double *B)
{
    double s = 0.0;
    for (int a = 0; a < c->dim; ++a) {
        int e = c->L.e[j][a];
        if (e == 1) s = s + B[a];
        else if (e == -1) s = s - B[a];
    }
    return s;
}

static int make_ctx(const orc_params *P, orc_ctx *c)
{
    memset(c, 0, sizeof(*c));
    /* per-axis d0 and spacing (rectangular lattice: linear CDE only) */
    double d0v[3] = {P->d0, P->d0, P->d0}, dxv[3] = {P->dx, P->dx, P->dx};
    if (P->rect) {
        if (P->eq != ORC_LCDE) return -1;
        for (int a = 0; a < 3; ++a) { d0v[a] = P->d0v[a]; dxv[a] = P->dxv[a]; }
    }
    if (build_lattice_v(P->lattice, d0v, &c->L)) return -1;
    c->rect = P->rect;
    for (int a = 0; a < 3; ++a) c->inv_d0v[a] = 1.0 / d0v[a];
    c->dim = c->L.dim;
    c->N = 1;
    for (int a = 0; a < 3; ++a) {
        c->n[a] = a < c->dim ? P->n[a] : 1;
        if (c->n[a] < 1) return -2;
        c->N *= c->n[a];
    }
    const double d0 = P->d0;
    c->inv_d0 = 1.0 / d0;
    /* Eq. (3-4) in lattice units: c~_ja = e_ja / d0_a,
     * Q~_jaa = (e_ja^2 - d0_a) / (d0_a (1 - d0_a)), Q~_jab = e_ja e_jb / (2 d0_a d0_b)
     * (the factor 2 of the off-diagonal pair is taken by summing (a,b) once) */
    for (int j = 0; j < c->L.b; ++j) {
        for (int a = 0; a < 3; ++a) {
            double ea = (double)c->L.e[j][a];
            c->qd[j][a] = (ea * ea - d0v[a]) / (d0v[a] * (1.0 - d0v[a]));
        }
        for (int o = 0; o < 3; ++o)
            c->qo[j][o] = (double)(c->L.e[j][OFF_A[o]] * c->L.e[j][OFF_B[o]]) /
                          (d0v[OFF_A[o]] * d0v[OFF_B[o]]);
        c->w1[j] = c->L.w[j] * c->inv_d0;
    }
    /* scheme sums, Eq. (2-7-1) */
    c->A0 = P->a[0] + P->a[1] + P->a[2];
    c->Ah0 = P->ah[0] + P->ah[1] + P->ah[2];
    c->Ab0 = P->ab[0] + P->ab[1] + P->ab[2];
    c->Abh0 = P->abh[0] + P->abh[1] + P->abh[2];
    c->ap = P->a[2] + P->a[0];    c->am = P->a[2] - P->a[0];
    c->ahp = P->ah[2] + P->ah[0]; c->ahm = P->ah[2] - P->ah[0];
    if (P->multiset) {
        /* Eq. (2-2-1b): the even parts' second differences take the even
         * set, the odd parts' first differences the odd set */
        if (P->eq == ORC_NSE) return -4;
        c->ap = P->ae[2] + P->ae[0];    c->am = P->ao[2] - P->ao[0];
        c->ahp = P->aeh[2] + P->aeh[0]; c->ahm = P->aoh[2] - P->aoh[0];
    }
    c->abp = P->ab[2] + P->ab[0]; c->abm = P->ab[2] - P->ab[0];
    c->abhp = P->abh[2] + P->abh[0]; c->abhm = P->abh[2] - P->abh[0];

    if (P->eq == ORC_LCDE) {
        /* Eq. (4-2-00a): A10 = -(ah sum) - 1, A22 = (a+ + ah+)/2; the EDF
         * diffusion tensor follows alpha = -(A22/A10) dt beta c_s^2. */
        double A10 = -c->Ah0 - 1.0;
        double A22 = 0.5 * (c->ap + c->ahp);
        double ratio = P->ratio > 0.0 ? P->ratio : -A10 / A22;
        /* lattice units per axis: u_a dt / dx_a, K_ab dt / (dx_a dx_b) */
        for (int a = 0; a < 3; ++a) c->uh[a] = P->u[a] * P->dt / dxv[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                c->kh[a * 3 + b] = P->K[a * 3 + b] * P->dt / (dxv[a] * dxv[b]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = ratio * c->kh[a * 3 + b];
                if (a == b) v = v - d0v[a];
                if (P->lambda_bar) v = v + c->uh[a] * c->uh[b];
                c->Ch[a * 3 + b] = v;
            }
        /* c~_j . uh: e_ja uh_a / d0_a summed over the axes (square: one d0) */
        double ut[3];
        for (int a = 0; a < 3; ++a) ut[a] = c->uh[a] / d0v[a];
        for (int j = 0; j < c->L.b; ++j) {
            double lin = P->rect ? edot(c, j, ut) : edot(c, j, c->uh) * c->inv_d0;
            c->ubar[j] = c->L.w[j] * ((1.0 + lin) + quad_term(c, j, c->Ch));
        }
        for (int p = 0; p < c->L.npair; ++p) {
            int j = c->L.pair[p];
            c->ubp[p] = c->L.w[j] * (1.0 + quad_term(c, j, c->Ch));
            c->ubm[p] = P->rect ? c->L.w[j] * edot(c, j, ut) : c->w1[j] * edot(c, j, c->uh);
            c->Cp[p] = c->ap * c->ubp[p];
            c->Cm[p] = c->am * c->ubm[p];
            c->Chp[p] = c->ahp * c->ubp[p];
            c->Chm[p] = c->ahm * c->ubm[p];
        }
    } else if (P->eq == ORC_WAVE) {
        /* Example 3: f_j = w_j phi [1 + (beta-1)(|e_j|^2 - dim d0)/(2 d0)],
         * the EDF printed there (its 2 c_s^2 is dim c_s^2 for dim = 2); a
         * linear EDF with no odd part */
        for (int j = 0; j < c->L.b; ++j) {
            double e2 = 0.0;
            for (int a = 0; a < 3; ++a) e2 = e2 + (double)(c->L.e[j][a] * c->L.e[j][a]);
            double t = (e2 - (double)c->dim * d0) / (2.0 * d0);
            c->ubar[j] = c->L.w[j] * (1.0 + (P->beta - 1.0) * t);
        }
        for (int p = 0; p < c->L.npair; ++p) {
            int j = c->L.pair[p];
            c->ubp[p] = c->ubar[j];
            c->ubm[p] = 0.0;
            c->Cp[p] = c->ap * c->ubp[p];
            c->Cm[p] = 0.0;
            c->Chp[p] = c->ahp * c->ubp[p];
            c->Chm[p] = 0.0;
        }
    } else if (P->eq == ORC_BURGERS) {
        c->bh = 0.5 * P->dt / P->dx;
        c->beta_one = P->beta == 1.0;
        c->cbeta = (P->beta - 1.0) * d0;
    } else if (P->eq == ORC_NSE) {
        c->rho0 = P->rho0;
        c->he_luo = P->he_luo;
        c->rinv0 = 1.0 / P->rho0;
    } else {
        return -3;
    }
    return 0;
}

/* ------------------------------------------------------------ grid helpers */

static inline int64_t wrap(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* index of node (x,y,z) shifted by k*e_j, periodic */
static inline int64_t nb(const orc_ctx *c, int64_t x, int64_t y, int64_t z, int j, int k)
{
    int64_t xs = wrap(x + k * c->L.e[j][0], c->n[0]);
    int64_t ys = wrap(y + k * c->L.e[j][1], c->n[1]);
    int64_t zs = wrap(z + k * c->L.e[j][2], c->n[2]);
    return (zs * c->n[1] + ys) * c->n[0] + xs;
}

static int nfields(const orc_params *P, const orc_ctx *c)
{
    return P->eq == ORC_NSE ? 1 + c->dim : 1;
}

/* EDF arguments (A, B, C) at one node from its moments m[0..nf-1] */
static void edf_args(const orc_ctx *c, int eq, const double *m, double *A,
                     double B[3], double C[9], int *hasC)
{
    memset(C, 0, 9 * sizeof(double));
    B[0] = B[1] = B[2] = 0.0;
    *A = m[0];
    *hasC = 1;
    if (eq == ORC_BURGERS) {
        double bh = (m[0] * m[0]) * c->bh;
        for (int a = 0; a < c->dim; ++a) B[a] = bh;
        if (c->beta_one) {
            *hasC = 0;
        } else {
            for (int a = 0; a < c->dim; ++a) C[a * 3 + a] = c->cbeta * m[0];
        }
    } else { /* NSE: A = rho - rho0, B = j, C = j j / rho */
        double r = c->he_luo ? c->rinv0 : 1.0 / (c->rho0 + m[0]);
        for (int a = 0; a < c->dim; ++a) B[a] = m[1 + a];
        for (int a = 0; a < c->dim; ++a)
            for (int b = 0; b < c->dim; ++b)
                C[a * 3 + b] = (B[a] * B[b]) * r;
    }
}

/* full EDF g_j(A,B,C), Eq. (3-3) */
static double edf_full(const orc_ctx *c, int j, double A, const double *B,
                       const double *C, int hasC)
{
    double t;
    if (c->rect) {
        double Bt[3];
        for (int a = 0; a < 3; ++a) Bt[a] = B[a] * c->inv_d0v[a];
        t = A + edot(c, j, Bt);
    } else {
        t = A + edot(c, j, B) * c->inv_d0;
    }
    if (hasC) t = t + quad_term(c, j, C);
    return c->L.w[j] * t;
}

/* ------------------------------------------------------------------- MMFD */

static double d2(const double *g, int64_t ip, int64_t i0, int64_t im)
{
    return (g[ip] - 2.0 * g[i0]) + g[im];
}

static double d1(const double *g, int64_t ip, int64_t im)
{
    return g[ip] - g[im];
}

/* even / odd pair EDF parts of one level over the whole grid:
 * Fp[p*N + i] = w_p (A + Q_p:C),  Fm[p*N + i] = (w_p/d0) e_p.B              */
static void pair_parts(const orc_params *P, const orc_ctx *c, const double *lev,
                       double *Fp, double *Fm)
{
    const int64_t N = c->N;
    const int nf = nfields(P, c);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double m[4], A, B[3], C[9];
        int hasC;
        for (int f = 0; f < nf; ++f) m[f] = lev[f * N + i];
        edf_args(c, P->eq, m, &A, B, C, &hasC);
        for (int p = 0; p < c->L.npair; ++p) {
            int j = c->L.pair[p];
            double t = A;
            if (hasC) t = t + quad_term(c, j, C);
            Fp[p * N + i] = c->L.w[j] * t;
            Fm[p * N + i] = c->w1[j] * edot(c, j, B);
        }
    }
}

/*
 * One MMFD step, central form Eq. (2-2-1) / (2-4-1), three-level form
 * Eq. (3layerMMFD-2); the LCDE uses the linear pair form Eq. (LMMFD-1/3)
 * with the constants (a_1 +- a_-1) ubar+-_p folded per pair.
 *   cur  : level t      (nf fields, field-major)
 *   prev : level t - dt (ignored for two-level)
 *   out  : level t + dt
 */
static int mmfd_step_all(const orc_params *P, const double *cur, const double *prev, double *out);
static int literal_step_all(const orc_params *P, const double *cur, const double *prev,
                            double *out);

static int is_linear(const orc_params *P) { return P->eq == ORC_LCDE || P->eq == ORC_WAVE; }

/* Dirichlet edges (2D scalar equations only) */
static int bc_ok(const orc_params *P, const orc_ctx *c)
{
    if (!P->bc) return 1;
    return c->dim == 2 && P->eq != ORC_NSE && P->bG != NULL;
}

/* the edge nodes of a new level take their prescribed values */
static void apply_dirichlet(const orc_params *P, const orc_ctx *c, double *out)
{
    for (int64_t y = 0; y < c->n[1]; ++y)
        for (int64_t x = 0; x < c->n[0]; ++x) {
            if (!(x == 0 || y == 0 || x == c->n[0] - 1 || y == c->n[1] - 1)) continue;
            int64_t i = y * c->n[0] + x;
            out[i] = P->bG[i] * P->bscale;
        }
}

int orc_mmfd_step(const orc_params *P, const double *cur, const double *prev, double *out)
{
    orc_ctx c;
    if (make_ctx(P, &c) || !bc_ok(P, &c)) return -1;
    int rc = mmfd_step_all(P, cur, prev, out);
    if (rc == 0 && P->bc) apply_dirichlet(P, &c, out);
    return rc;
}

/* every node updated by the scheme (periodic wrap at the grid's edges) */
static int mmfd_step_all(const orc_params *P, const double *cur, const double *prev, double *out)
{
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    const int64_t N = c.N;
    const int three = P->levels == 3;
    const int np = c.L.npair;

    if (is_linear(P)) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int64_t z = 0; z < c.n[2]; ++z)
            for (int64_t y = 0; y < c.n[1]; ++y)
                for (int64_t x = 0; x < c.n[0]; ++x) {
                    int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                    double acc = 0.0;
                    for (int p = 0; p < np; ++p) {
                        int j = c.L.pair[p];
                        int64_t ip = nb(&c, x, y, z, j, 1), im = nb(&c, x, y, z, j, -1);
                        acc = acc + c.Cp[p] * d2(cur, ip, i, im);
                        acc = acc + c.Cm[p] * d1(cur, ip, im);
                    }
                    if (three) {
                        for (int p = 0; p < np; ++p) {
                            int j = c.L.pair[p];
                            int64_t ip = nb(&c, x, y, z, j, 1), im = nb(&c, x, y, z, j, -1);
                            acc = acc + c.Chp[p] * d2(prev, ip, i, im);
                            acc = acc + c.Chm[p] * d1(prev, ip, im);
                        }
                    }
                    double base = c.A0 * cur[i];
                    if (three) base = base + c.Ah0 * prev[i];
                    out[i] = base + acc;
                }
        return 0;
    }

    /* nonlinear EDFs: pair parts of each level, then central differences */
    double *Fp = malloc(sizeof(double) * np * N), *Fm = malloc(sizeof(double) * np * N);
    double *Hp = NULL, *Hm = NULL;
    if (!Fp || !Fm) { free(Fp); free(Fm); return -4; }
    pair_parts(P, &c, cur, Fp, Fm);
    /* a level-(t-dt) stencil exists only if one of its pair sums is nonzero;
     * skipping an all-zero term leaves every finite value unchanged */
    const int three_st = three && (c.ahp != 0.0 || c.ahm != 0.0 ||
                                   c.abhp != 0.0 || c.abhm != 0.0);
    if (three_st) {
        Hp = malloc(sizeof(double) * np * N);
        Hm = malloc(sizeof(double) * np * N);
        if (!Hp || !Hm) { free(Fp); free(Fm); free(Hp); free(Hm); return -4; }
        pair_parts(P, &c, prev, Hp, Hm);
    }
    const int nf = nfields(P, &c);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c.n[2]; ++z)
        for (int64_t y = 0; y < c.n[1]; ++y)
            for (int64_t x = 0; x < c.n[0]; ++x) {
                int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                int64_t ip[ORC_MAXP], im[ORC_MAXP];
                for (int p = 0; p < np; ++p) {
                    ip[p] = nb(&c, x, y, z, c.L.pair[p], 1);
                    im[p] = nb(&c, x, y, z, c.L.pair[p], -1);
                }
                /* zeroth moment: a+ D2 F+ + a- D1 F- */
                double acc = 0.0;
                for (int p = 0; p < np; ++p) {
                    acc = acc + c.ap * d2(Fp + p * N, ip[p], i, im[p]);
                    acc = acc + c.am * d1(Fm + p * N, ip[p], im[p]);
                }
                if (three_st)
                    for (int p = 0; p < np; ++p) {
                        acc = acc + c.ahp * d2(Hp + p * N, ip[p], i, im[p]);
                        acc = acc + c.ahm * d1(Hm + p * N, ip[p], im[p]);
                    }
                double base = c.A0 * cur[i];
                if (three) base = base + c.Ah0 * prev[i];
                out[i] = base + acc;
                /* first moments (NSE): e_p [ab+ D2 F- + ab- D1 F+] */
                for (int f = 1; f < nf; ++f) {
                    int a = f - 1;
                    double m = 0.0;
                    for (int p = 0; p < np; ++p) {
                        int e = c.L.e[c.L.pair[p]][a];
                        if (e == 0) continue;
                        double t1 = c.abp * d2(Fm + p * N, ip[p], i, im[p]);
                        double t2 = c.abm * d1(Fp + p * N, ip[p], im[p]);
                        if (e == 1) { m = m + t1; m = m + t2; }
                        else        { m = m - t1; m = m - t2; }
                    }
                    if (three_st)
                        for (int p = 0; p < np; ++p) {
                            int e = c.L.e[c.L.pair[p]][a];
                            if (e == 0) continue;
                            double t1 = c.abhp * d2(Hm + p * N, ip[p], i, im[p]);
                            double t2 = c.abhm * d1(Hp + p * N, ip[p], im[p]);
                            if (e == 1) { m = m + t1; m = m + t2; }
                            else        { m = m - t1; m = m - t2; }
                        }
                    double bj = c.Ab0 * cur[f * N + i];
                    if (three) bj = bj + c.Abh0 * prev[f * N + i];
                    out[f * N + i] = bj + m;
                }
            }
    free(Fp); free(Fm); free(Hp); free(Hm);
    return 0;
}

/* ----------------------------------------------------------------- LITERAL */

/* full EDF of every direction of one level over the grid: G[j*N + i] */
static void full_edf(const orc_params *P, const orc_ctx *c, const double *lev, double *G)
{
    const int64_t N = c->N;
    const int nf = nfields(P, c);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if (is_linear(P)) {
            for (int j = 0; j < c->L.b; ++j) G[j * N + i] = c->ubar[j] * lev[i];
            continue;
        }
        double m[4], A, B[3], C[9];
        int hasC;
        for (int f = 0; f < nf; ++f) m[f] = lev[f * N + i];
        edf_args(c, P->eq, m, &A, B, C, &hasC);
        for (int j = 0; j < c->L.b; ++j) G[j * N + i] = edf_full(c, j, A, B, C, hasC);
    }
}

/*
 * The scheme taken literally, Eqs. (2-2)/(2-3)/(2-4)/(3layerMMFD-1):
 *   phi(x, t+dt) = sum_j sum_(k,level) a_k f_j^eq(x + k e_j, level)
 * and for the NSE first moments the same with e_j and the momentum set.
 */
/*
 * Population j at node (x,y,z) of the multiple-set scheme, Eq. (2-1b):
 *   f_j = sum_k [ ae_k g+_j(x + k e_j) + ao_k g-_j(x + k e_j) ]   (level t)
 *       + sum_k [ aeh_k g+_j(...) + aoh_k g-_j(...) ]              (level t - dt)
 * with g+-_j = (g_j +- g_jbar)/2 the even / odd parts of the EDF at the same
 * node (Eq. (2-5)); zero coefficients skipped, k = -1, 0, +1, level t first.
 */
static double multiset_pop(const orc_params *P, const orc_ctx *c, const double *G,
                           const double *H, int j, int64_t x, int64_t y, int64_t z)
{
    const int64_t N = c->N;
    const int jb = c->L.opp[j];
    double fj = 0.0;
    for (int lev = 0; lev < (H ? 2 : 1); ++lev) {
        const double *L = lev == 0 ? G : H;
        const double *ae = lev == 0 ? P->ae : P->aeh, *ao = lev == 0 ? P->ao : P->aoh;
        for (int k = -1; k <= 1; ++k) {
            int64_t y0 = nb(c, x, y, z, j, k);
            double gp = 0.5 * (L[j * N + y0] + L[jb * N + y0]);
            double gm = 0.5 * (L[j * N + y0] - L[jb * N + y0]);
            if (ae[k + 1] != 0.0) fj = fj + ae[k + 1] * gp;
            if (ao[k + 1] != 0.0) fj = fj + ao[k + 1] * gm;
        }
    }
    return fj;
}

int orc_literal_step(const orc_params *P, const double *cur, const double *prev, double *out)
{
    orc_ctx c;
    if (make_ctx(P, &c) || !bc_ok(P, &c)) return -1;
    int rc = literal_step_all(P, cur, prev, out);
    if (rc == 0 && P->bc) apply_dirichlet(P, &c, out);
    return rc;
}

static int literal_step_all(const orc_params *P, const double *cur, const double *prev,
                            double *out)
{
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    const int64_t N = c.N;
    const int three = P->levels == 3;
    const int b = c.L.b;
    const int nf = nfields(P, &c);
    double *G = malloc(sizeof(double) * b * N), *H = NULL;
    if (!G) return -4;
    full_edf(P, &c, cur, G);
    if (three) {
        H = malloc(sizeof(double) * b * N);
        if (!H) { free(G); return -4; }
        full_edf(P, &c, prev, H);
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c.n[2]; ++z)
        for (int64_t y = 0; y < c.n[1]; ++y)
            for (int64_t x = 0; x < c.n[0]; ++x) {
                int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                for (int f = 0; f < nf; ++f) {
                    const double *ak = f == 0 ? P->a : P->ab;
                    const double *ahk = f == 0 ? P->ah : P->abh;
                    double s = 0.0;
                    for (int j = 0; j < b; ++j) {
                        int e = f == 0 ? 1 : c.L.e[j][f - 1];
                        if (e == 0) continue;
                        double fj = 0.0;
                        if (P->multiset) {
                            fj = multiset_pop(P, &c, G, three ? H : NULL, j, x, y, z);
                        } else {
                            for (int k = -1; k <= 1; ++k)
                                if (ak[k + 1] != 0.0) fj = fj + ak[k + 1] * G[j * N + nb(&c, x, y, z, j, k)];
                            if (three)
                                for (int k = -1; k <= 1; ++k)
                                    if (ahk[k + 1] != 0.0) fj = fj + ahk[k + 1] * H[j * N + nb(&c, x, y, z, j, k)];
                        }
                        s = e == 1 ? s + fj : s - fj;
                    }
                    out[f * N + i] = s;
                }
            }
    free(G); free(H);
    return 0;
}

/* ------------------------------------------------------------ source term */

/*
 * Source of the scheme, the b terms of Eq. (2-1) / (3layerMMFD-1):
 *   Delta t sum_j sum_k [ b_k F_j(x + k e_j, t) + bh_k F_j(x + k e_j, t - dt) ]
 * with F_j of Eq. (SourceF) for the NCDE: F_j = w_j (S + c_j.M_1F / c_s^2),
 * M_1F = v S for a constant vector v, i.e. in lattice units
 *   F_j(y) = w_j (S(y) + (e_j.vh / d0) S(y)),   vh = v dt / dx.
 * S is given at both time levels (the caller evaluates it); its time levels
 * are independent of the scheme's levels of phi.
 */
typedef struct {
    double b[3], bh[3];   /* k = -1, 0, +1 at level t and t - dt            */
    double v[3];          /* M_1F = v S (physical velocity)                 */
} orc_source;

/* the source term of direction j at node (x, y, z), before the factor dt:
 *   sum_k b_k F_j(x + k e_j, t) + sum_k bh_k F_j(x + k e_j, t - dt),
 * zero coefficients skipped, level t first */
static double source_dir(const orc_params *P, const orc_ctx *c, const orc_source *Q,
                         const double *St, const double *Sm, int j, int64_t x, int64_t y,
                         int64_t z)
{
    double vh[3];
    for (int a = 0; a < 3; ++a) vh[a] = Q->v[a] * P->dt / P->dx;
    double ev = edot(c, j, vh) * c->inv_d0;
    double sj = 0.0;
    for (int lev = 0; lev < 2; ++lev) {
        const double *S = lev == 0 ? St : Sm;
        const double *bk = lev == 0 ? Q->b : Q->bh;
        for (int k = -1; k <= 1; ++k) {
            if (bk[k + 1] == 0.0) continue;
            double Sy = S[nb(c, x, y, z, j, k)];
            sj = sj + bk[k + 1] * (c->L.w[j] * (Sy + ev * Sy));
        }
    }
    return sj;
}



/* ------------------------------------------------------------------ MesoFD */

/* populations of the EDF of a moment state: pop[j*N + i] = f_j^eq(i) */
int orc_init_populations(const orc_params *P, const double *mom, double *pop)
{
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    full_edf(P, &c, mom, pop);
    return 0;
}

/* moments of populations, Eq. (2-1-1): phi = sum_j f_j, j = sum_j e_j f_j */
int orc_moments(const orc_params *P, const double *pop, double *mom)
{
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    const int64_t N = c.N;
    const int nf = nfields(P, &c);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        for (int f = 0; f < nf; ++f) {
            double s = 0.0;
            for (int j = 0; j < c.L.b; ++j) {
                int e = f == 0 ? 1 : c.L.e[j][f - 1];
                if (e == 1) s = s + pop[j * N + i];
                else if (e == -1) s = s - pop[j * N + i];
            }
            mom[f * N + i] = s;
        }
    }
    return 0;
}

/*
 * One MesoFD step, Eq. (2-1) / (3layer-1):
 *   f_j(x, t+dt) = sum_k a_k f_j^eq(x + k e_j, t) + sum_k ah_k f_j^eq(x + k e_j, t-dt)
 * with f^eq at level t built from the moments of the populations `pop` and
 * at level t-dt from the stored moments `prev_mom` (three-level only).
 * Writes the new populations and, for three-level schemes, the moments of
 * level t (the t-dt level of the next step) into `mom_out`.
 */
static int mesofd_step(const orc_params *P, const orc_source *Q, const double *pop,
                       const double *prev_mom, const double *St, const double *Sm,
                       double *pop_out, double *mom_out);

int orc_mesofd_step(const orc_params *P, const double *pop, const double *prev_mom,
                    double *pop_out, double *mom_out)
{
    return mesofd_step(P, NULL, pop, prev_mom, NULL, NULL, pop_out, mom_out);
}

/* the populations of one step, Eq. (2-1) / (3layer-1), with the source
 * term of each direction added when Q is given */
static int mesofd_step(const orc_params *P, const orc_source *Q, const double *pop,
                       const double *prev_mom, const double *St, const double *Sm,
                       double *pop_out, double *mom_out)
{
    orc_ctx c;
    if (make_ctx(P, &c) || P->bc) return -1;  /* MesoFD: periodic grids */
    const int64_t N = c.N;
    const int b = c.L.b;
    const int nf = nfields(P, &c);
    const int three = P->levels == 3;
    double *mom = malloc(sizeof(double) * nf * N);
    double *G = malloc(sizeof(double) * b * N), *H = NULL;
    if (!mom || !G) { free(mom); free(G); return -4; }
    orc_moments(P, pop, mom);
    full_edf(P, &c, mom, G);
    if (three) {
        H = malloc(sizeof(double) * b * N);
        if (!H) { free(mom); free(G); return -4; }
        full_edf(P, &c, prev_mom, H);
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c.n[2]; ++z)
        for (int64_t y = 0; y < c.n[1]; ++y)
            for (int64_t x = 0; x < c.n[0]; ++x) {
                int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                for (int j = 0; j < b; ++j) {
                    double fj = 0.0;
                    if (P->multiset) {
                        fj = multiset_pop(P, &c, G, three ? H : NULL, j, x, y, z);
                    } else {
                        for (int k = -1; k <= 1; ++k)
                            if (P->a[k + 1] != 0.0) fj = fj + P->a[k + 1] * G[j * N + nb(&c, x, y, z, j, k)];
                        if (three)
                            for (int k = -1; k <= 1; ++k)
                                if (P->ah[k + 1] != 0.0) fj = fj + P->ah[k + 1] * H[j * N + nb(&c, x, y, z, j, k)];
                    }
                    if (Q) fj = fj + P->dt * source_dir(P, &c, Q, St, Sm, j, x, y, z);
                    pop_out[j * N + i] = fj;
                }
            }
    if (mom_out) memcpy(mom_out, mom, sizeof(double) * nf * N);
    free(mom); free(G); free(H);
    return 0;
}

double orc_sum(const double *v, int64_t n);

/* --------------------------------------------------------- theta (linear) */

/*
 * Two-level theta scheme for the LCDE, Eq. (GCN):
 *   (I - (1-theta) L) phi(t+dt) = (A0 I + theta L) phi(t),   A0 = sum_k a_k,
 * L = the explicit increment of Eq. (LMMFD-3).  Solved by `theta_iters`
 * Jacobi sweeps started from phi(t).
 */
int orc_theta_step(const orc_params *P, const double *cur, double *out, double *work)
{
    orc_ctx c;
    if (make_ctx(P, &c) || P->eq != ORC_LCDE || P->bc) return -1;
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    const int64_t N = c.N;
    const int np = c.L.npair;
    const double th = P->theta, th1 = 1.0 - P->theta;
    double sp = 0.0;
    for (int p = 0; p < np; ++p) sp = sp + c.Cp[p];
    const double inv_den = 1.0 / (1.0 + th1 * (2.0 * sp));
    double *rhs = malloc(sizeof(double) * N);
    if (!rhs) return -4;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c.n[2]; ++z)
        for (int64_t y = 0; y < c.n[1]; ++y)
            for (int64_t x = 0; x < c.n[0]; ++x) {
                int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                double acc = 0.0;
                for (int p = 0; p < np; ++p) {
                    int j = c.L.pair[p];
                    int64_t ip = nb(&c, x, y, z, j, 1), im = nb(&c, x, y, z, j, -1);
                    acc = acc + c.Cp[p] * d2(cur, ip, i, im);
                    acc = acc + c.Cm[p] * d1(cur, ip, im);
                }
                rhs[i] = c.A0 * cur[i] + th * acc;
            }
    /* Jacobi sweeps, iterate k in `work` / `out` alternately, ends in out */
    const double *src = cur;
    for (int it = 0; it < P->theta_iters; ++it) {
        double *dst = ((P->theta_iters - it) % 2 == 1) ? out : work;
#pragma omp parallel for collapse(2) schedule(static)
        for (int64_t z = 0; z < c.n[2]; ++z)
            for (int64_t y = 0; y < c.n[1]; ++y)
                for (int64_t x = 0; x < c.n[0]; ++x) {
                    int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                    double acc = 0.0;
                    for (int p = 0; p < np; ++p) {
                        int j = c.L.pair[p];
                        int64_t ip = nb(&c, x, y, z, j, 1), im = nb(&c, x, y, z, j, -1);
                        acc = acc + c.Cp[p] * (src[ip] + src[im]);
                        acc = acc + c.Cm[p] * (src[ip] - src[im]);
                    }
                    dst[i] = (rhs[i] + th1 * acc) * inv_den;
                }
        src = dst;
    }
    if (P->theta_iters == 0) memcpy(out, cur, sizeof(double) * N);
    free(rhs);
    return 0;
}

/*
 * The same theta step solved to a tolerance: Jacobi sweeps (as above, started
 * from phi(t)) in chunks of `chunk` sweeps; after each chunk the residual of
 * the iterate before the chunk's last sweep is
 *     r = rhs - (I - (1-theta) L) x_{k-1} = den (x_k - x_{k-1}),
 *     den = 1 + (1-theta) 2 sum_p Cp_p
 * (the Jacobi update written out), and the solve stops at the first chunk
 * with  den^2 sum (x_k - x_{k-1})^2 <= tol^2 sum rhs^2  (both sums
 * compensated), or when `cap` sweeps are reached.  Returns x_k in `out`, the
 * sweeps taken in *sweeps and 1 / 0 in *converged.
 */
int orc_theta_solve(const orc_params *P, const double *cur, double *out, double *work,
                    double tol, int chunk, int cap, int *sweeps, int *converged)
{
    orc_ctx c;
    if (make_ctx(P, &c) || P->eq != ORC_LCDE || P->bc || chunk < 1 || cap < 1) return -1;
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    const int64_t N = c.N;
    const int np = c.L.npair;
    const double th = P->theta, th1 = 1.0 - P->theta;
    double sp = 0.0;
    for (int p = 0; p < np; ++p) sp = sp + c.Cp[p];
    const double den = 1.0 + th1 * (2.0 * sp);
    const double inv_den = 1.0 / den;
    double *rhs = malloc(sizeof(double) * N), *sq = malloc(sizeof(double) * N);
    double *x[2] = {out, work};
    if (!rhs || !sq) { free(rhs); free(sq); return -4; }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c.n[2]; ++z)
        for (int64_t y = 0; y < c.n[1]; ++y)
            for (int64_t xx = 0; xx < c.n[0]; ++xx) {
                int64_t i = (z * c.n[1] + y) * c.n[0] + xx;
                double acc = 0.0;
                for (int p = 0; p < np; ++p) {
                    int j = c.L.pair[p];
                    int64_t ip = nb(&c, xx, y, z, j, 1), im = nb(&c, xx, y, z, j, -1);
                    acc = acc + c.Cp[p] * d2(cur, ip, i, im);
                    acc = acc + c.Cm[p] * d1(cur, ip, im);
                }
                rhs[i] = c.A0 * cur[i] + th * acc;
            }
    for (int64_t i = 0; i < N; ++i) sq[i] = rhs[i] * rhs[i];
    const double b2 = orc_sum(sq, N);
    const double *src = cur;
    int k = 0, done = 0, conv = 0, w = 0;
    while (!done) {
        for (int it = 0; it < chunk; ++it) {
            double *dst = x[w];
#pragma omp parallel for collapse(2) schedule(static)
            for (int64_t z = 0; z < c.n[2]; ++z)
                for (int64_t y = 0; y < c.n[1]; ++y)
                    for (int64_t xx = 0; xx < c.n[0]; ++xx) {
                        int64_t i = (z * c.n[1] + y) * c.n[0] + xx;
                        double acc = 0.0;
                        for (int p = 0; p < np; ++p) {
                            int j = c.L.pair[p];
                            int64_t ip = nb(&c, xx, y, z, j, 1), im = nb(&c, xx, y, z, j, -1);
                            acc = acc + c.Cp[p] * (src[ip] + src[im]);
                            acc = acc + c.Cm[p] * (src[ip] - src[im]);
                        }
                        dst[i] = (rhs[i] + th1 * acc) * inv_den;
                    }
            ++k;
            if (it + 1 == chunk) {
                for (int64_t i = 0; i < N; ++i) {
                    double d = dst[i] - src[i];
                    sq[i] = d * d;
                }
            }
            src = dst;
            w ^= 1;
        }
        const double d2s = orc_sum(sq, N);
        conv = den * den * d2s <= tol * tol * b2;
        done = conv || k >= cap;
    }
    if (src != out) memcpy(out, src, sizeof(double) * N);
    *sweeps = k;
    *converged = conv;
    free(rhs); free(sq);
    return 0;
}

/* MMFD form: Eq. (2-2-1) with its b terms,
 *   dt [ B0 S(t) + Bh0 S(t-dt) ]
 *   + dt sum_p [ b+ D2_p F+(t) + b- D1_p F-(t) + bh+ D2_p F+(t-dt) + bh- D1_p F-(t-dt) ]
 * with B0 = sum_k b_k, b+- = b_1 +- b_-1, the pair parts F+_p = w_p S and
 * F-_p = (w_p / d0)(e_p.vh) S (the even / odd split of Eq. (2-5)), every pair
 * counted once for both of its directions. */
static void source_mmfd(const orc_params *P, const orc_ctx *c, const orc_source *Q,
                        const double *St, const double *Sm, double *out)
{
    double vh[3];
    for (int a = 0; a < 3; ++a) vh[a] = Q->v[a] * P->dt / P->dx;
    const int np = c->L.npair;
    double wp[ORC_MAXP], wm[ORC_MAXP];
    for (int p = 0; p < np; ++p) {
        int j = c->L.pair[p];
        wp[p] = c->L.w[j];
        wm[p] = c->w1[j] * edot(c, j, vh);
    }
    const double B0 = Q->b[0] + Q->b[1] + Q->b[2];
    const double Bh0 = Q->bh[0] + Q->bh[1] + Q->bh[2];
    const double bp = Q->b[2] + Q->b[0], bm = Q->b[2] - Q->b[0];
    const double bhp = Q->bh[2] + Q->bh[0], bhm = Q->bh[2] - Q->bh[0];
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c->n[2]; ++z)
        for (int64_t y = 0; y < c->n[1]; ++y)
            for (int64_t x = 0; x < c->n[0]; ++x) {
                int64_t i = (z * c->n[1] + y) * c->n[0] + x;
                double sv = B0 * St[i] + Bh0 * Sm[i];
                double sa = 0.0;
                for (int lev = 0; lev < 2; ++lev) {
                    const double *S = lev == 0 ? St : Sm;
                    const double cp = lev == 0 ? bp : bhp, cm = lev == 0 ? bm : bhm;
                    for (int p = 0; p < np; ++p) {
                        int j = c->L.pair[p];
                        int64_t ip = nb(c, x, y, z, j, 1), im = nb(c, x, y, z, j, -1);
                        double d2v = (wp[p] * S[ip] - 2.0 * (wp[p] * S[i])) + wp[p] * S[im];
                        double d1v = wm[p] * S[ip] - wm[p] * S[im];
                        sa = sa + cp * d2v;
                        sa = sa + cm * d1v;
                    }
                }
                out[i] = out[i] + P->dt * (sv + sa);
            }
}

/* one MMFD step of the linear CDE with the source: the step of
 * orc_mmfd_step, then its source term added */
int orc_mmfd_source_step(const orc_params *P, const orc_source *Q, const double *cur,
                         const double *prev, const double *St, const double *Sm, double *out)
{
    if (P->rect) return -1;  /* the source term is written for square lattices */
    if (P->eq != ORC_LCDE || P->bc) return -5;
    int rc = orc_mmfd_step(P, cur, prev, out);
    if (rc) return rc;
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
    source_mmfd(P, &c, Q, St, Sm, out);
    return 0;
}

/* the literal form: orc_literal_step, then
 *   dt sum_j sum_k [ b_k F_j(x + k e_j, t) + bh_k F_j(x + k e_j, t - dt) ]
 * with F_j evaluated direction by direction */
int orc_literal_source_step(const orc_params *P, const orc_source *Q, const double *cur,
                            const double *prev, const double *St, const double *Sm, double *out)
{
    if (P->rect) return -1;  /* the source term is written for square lattices */
    if (P->eq != ORC_LCDE || P->bc) return -5;
    int rc = orc_literal_step(P, cur, prev, out);
    if (rc) return rc;
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
    const int b = c.L.b;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c.n[2]; ++z)
        for (int64_t y = 0; y < c.n[1]; ++y)
            for (int64_t x = 0; x < c.n[0]; ++x) {
                int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                double s = 0.0;
                for (int j = 0; j < b; ++j) s = s + source_dir(P, &c, Q, St, Sm, j, x, y, z);
                out[i] = out[i] + P->dt * s;
            }
    return 0;
}

/* one MesoFD step of the linear CDE with the source: every population gets
 * dt times its direction's source term (source_dir) after its a terms */
int orc_mesofd_source_step(const orc_params *P, const orc_source *Q, const double *pop,
                           const double *prev_mom, const double *St, const double *Sm,
                           double *pop_out, double *mom_out)
{
    if (P->rect) return -1;  /* the source term is written for square lattices */
    if (P->eq != ORC_LCDE || P->bc) return -5;
    return mesofd_step(P, Q, pop, prev_mom, St, Sm, pop_out, mom_out);
}

/* ------------------------------------------------------- wave first step */

/*
 * Special first step of the three-level wave scheme (Example 3): a Taylor
 * step with phi_tt = alpha Laplacian(phi), alpha = A22 beta c_s^2
 * (Eq. (ME-NCDE-W-1)), the Laplacian by the axis second differences:
 *   phi(x, dt) = phi(x, 0) + dt phi_t(x, 0)
 *                + (dt^2 alpha / (2 dx^2)) sum_axes [phi(x+e_a) - 2 phi(x) + phi(x-e_a)]
 * whose factor is A22 beta d0 / 2 in lattice units (Example 3: (dt/(2dx))^2).
 * The wrap is periodic; with Dirichlet edges those nodes take bG * bscale
 * (bscale = exp(lambda dt)).
 */
int orc_wave_start(const orc_params *P, const double *phi0, const double *phit, double *out)
{
    orc_ctx c;
    if (make_ctx(P, &c) || P->eq != ORC_WAVE || P->levels != 3 || !bc_ok(P, &c)) return -1;
    const double A22 = 0.5 * (c.ap + c.ahp);
    const double cw = ((0.5 * A22) * P->beta) * P->d0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < c.n[2]; ++z)
        for (int64_t y = 0; y < c.n[1]; ++y)
            for (int64_t x = 0; x < c.n[0]; ++x) {
                int64_t i = (z * c.n[1] + y) * c.n[0] + x;
                double lap = 0.0;
                for (int a = 0; a < c.dim; ++a) {
                    int64_t xs[2] = {x, x}, ys[2] = {y, y}, zs[2] = {z, z};
                    if (a == 0) { xs[0] = wrap(x + 1, c.n[0]); xs[1] = wrap(x - 1, c.n[0]); }
                    if (a == 1) { ys[0] = wrap(y + 1, c.n[1]); ys[1] = wrap(y - 1, c.n[1]); }
                    if (a == 2) { zs[0] = wrap(z + 1, c.n[2]); zs[1] = wrap(z - 1, c.n[2]); }
                    int64_t ip = (zs[0] * c.n[1] + ys[0]) * c.n[0] + xs[0];
                    int64_t im = (zs[1] * c.n[1] + ys[1]) * c.n[0] + xs[1];
                    lap = lap + d2(phi0, ip, i, im);
                }
                out[i] = (phi0[i] + P->dt * phit[i]) + cw * lap;
            }
    if (P->bc) apply_dirichlet(P, &c, out);
    return 0;
}

/* ---------------------------------------------------------- tables / sums */

/* constant tables for cross-checks: w[b], ubar[b], ubp/ubm/Cp/Cm/Chp/Chm[np] */
int orc_tables(const orc_params *P, double *w, double *ubar, double *pairs6)
{
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
    for (int j = 0; j < c.L.b; ++j) {
        if (w) w[j] = c.L.w[j];
        if (ubar) ubar[j] = c.ubar[j];
    }
    if (pairs6)
        for (int p = 0; p < c.L.npair; ++p) {
            pairs6[0 * ORC_MAXP + p] = c.ubp[p];
            pairs6[1 * ORC_MAXP + p] = c.ubm[p];
            pairs6[2 * ORC_MAXP + p] = c.Cp[p];
            pairs6[3 * ORC_MAXP + p] = c.Cm[p];
            pairs6[4 * ORC_MAXP + p] = c.Chp[p];
            pairs6[5 * ORC_MAXP + p] = c.Chm[p];
        }
    return c.L.b;
}

/* lattice velocities (b x 3) and weights */
int orc_lattice_info(int lattice, double d0, int *e, double *w, int *npair, int *pairs)
{
    orc_lattice L;
    if (build_lattice(lattice, d0, &L)) return -1;
    for (int j = 0; j < L.b; ++j) {
        for (int a = 0; a < 3; ++a) e[j * 3 + a] = L.e[j][a];
        w[j] = L.w[j];
    }
    *npair = L.npair;
    for (int p = 0; p < L.npair; ++p) pairs[p] = L.pair[p];
    return L.b;
}

/* the same with d0_a per axis (rectangular lattices of Appendix A) */
int orc_lattice_info_rect(int lattice, const double *d0v, int *e, double *w, int *npair, int *pairs)
{
    orc_lattice L;
    if (build_lattice_v(lattice, d0v, &L)) return -1;
    for (int j = 0; j < L.b; ++j) {
        for (int a = 0; a < 3; ++a) e[j * 3 + a] = L.e[j][a];
        w[j] = L.w[j];
    }
    *npair = L.npair;
    for (int p = 0; p < L.npair; ++p) pairs[p] = L.pair[p];
    return L.b;
}

/* EDF g_j(A,B,C) of Eq. (3-3) for every direction (used by identity pins) */
int orc_edf(int lattice, double d0, double A, const double *B, const double *C, double *g)
{
    orc_params P;
    memset(&P, 0, sizeof(P));
    P.lattice = lattice; P.d0 = d0; P.eq = ORC_NSE; P.rho0 = 1.0;
    P.n[0] = P.n[1] = P.n[2] = 1;
    orc_ctx c;
    if (make_ctx(&P, &c)) return -1;
    for (int j = 0; j < c.L.b; ++j) g[j] = edf_full(&c, j, A, B, C, 1);
    return c.L.b;
}

/* the same on a rectangular lattice with d0_a per axis (c~_ja = e_ja / d0_a,
 * Q~ of Eq. (3-4) per axis) */
int orc_edf_rect(int lattice, const double *d0v, double A, const double *B, const double *C,
                 double *g)
{
    orc_params P;
    memset(&P, 0, sizeof(P));
    P.lattice = lattice; P.d0 = d0v[0]; P.eq = ORC_LCDE; P.rect = 1;
    P.dx = P.dt = 1.0;
    for (int a = 0; a < 3; ++a) { P.d0v[a] = d0v[a]; P.dxv[a] = 1.0; }
    P.n[0] = P.n[1] = P.n[2] = 1;
    orc_ctx c;
    if (make_ctx(&P, &c)) return -1;
    for (int j = 0; j < c.L.b; ++j) g[j] = edf_full(&c, j, A, B, C, 1);
    return c.L.b;
}

/* the pair parts F+_p, F-_p of every node of one level (Eq. (2-5) applied to
 * Eq. (3-3)), as the central form uses them: Fp[p * N + i], Fm[p * N + i] */
int orc_pair_parts(const orc_params *P, const double *lev, double *Fp, double *Fm)
{
    orc_ctx c;
    if (make_ctx(P, &c)) return -1;
    pair_parts(P, &c, lev, Fp, Fm);
    return c.L.npair;
}

/* Neumaier-compensated sum of n values */
double orc_sum(const double *v, int64_t n)
{
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i])) comp += (s - t) + v[i];
        else comp += (v[i] - t) + s;
        s = t;
    }
    return s + comp;
}
