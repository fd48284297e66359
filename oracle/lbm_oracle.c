/*
 * Plain CPU oracle for the double-distribution cascaded (central-moment,
 * multiple-relaxation-time) lattice Boltzmann method for 3D thermal
 * convection of Hajabdollahi & Premnath, "Central moments-based cascaded
 * lattice Boltzmann method for thermal convective flows in three dimensions"
 * (arXiv:1710.04751).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it and shares no code, table or header with it.
 *
 * Arithmetic is FP64 (`real` = double).  Building with -DORACLE_LONG_DOUBLE
 * gives the same code in x87 extended precision; comparing the two builds
 * measures the oracle's own rounding noise.
 *
 * How the oracle computes a collision.  The paper gives each cascaded kernel
 * (flow: Appendix A; thermal D3Q15: Sec. 2.2; thermal D3Q7: Appendix C) as a
 * closed-form algebraic result of one plain rule: relax every non-conserved
 * central moment, order by order, toward its equilibrium with its own rate,
 * keeping the conserved ones.  The oracle writes that rule out directly:
 *   1. central moments c_k = sum_a eta_a P_k(e_a - u) by direct summation;
 *   2. c~_k = c_k + omega_k (c_eq_k - c_k) for the relaxed ones;
 *   3. post-collision populations = the unique populations whose central
 *      moments about u are c~ (a dense linear solve with the matrix
 *      C_ka = P_k(e_a - u)).
 * The test suite checks that this equals the paper's printed kernels.
 *
 * Readings of points where the paper is silent or garbled are marked
 * "reading:" below and are listed in the design notes of the repository.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_LONG_DOUBLE
typedef long double real;
#define ORACLE_SYM(name) oracle_ld_##name
#else
typedef double real;
#define ORACLE_SYM(name) oracle_##name
#endif

#define QF 15 /* flow lattice: D3Q15 */
#define QMAX 15

/* ------------------------------------------------------------------------ */
/* Lattices                                                                   */
/* ------------------------------------------------------------------------ */

/* D3Q15 particle velocities in the order of Sec. 2.2, eq. (5): rest, the six
 * faces (+x,-x,+y,-y,+z,-z), then the eight corners. */
static const int E15[15][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 1},  {-1, 1, 1}, {1, -1, 1},
    {-1, -1, 1}, {1, 1, -1},  {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};

/* D3Q7 particle velocities in the order of Appendix C. */
static const int E7[7][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},
                             {0, -1, 0}, {0, 0, 1},  {0, 0, -1}};

/* Central-moment functionals P_k(c), c = e - u.
 *
 * 15-moment set (D3Q15, flow and thermal).  Orders follow the paper's
 * orthogonal basis K (Sec. 2.2) and the raw moments its kernels use
 * (Appendix A and the thermal kernel of Sec. 2.2):
 *   0: 1
 *   1..3: x, y, z
 *   4..6: xy, xz, yz
 *   7: xx-yy   8: xx+yy-2zz   9: xx+yy+zz
 *   10: xyy  11: xxy  12: xxz  13: xyz
 *   14: xxyy
 * 7-moment set (D3Q7, Appendix C): 1, x, y, z, xx-yy, xx+yy-2zz, xx+yy+zz. */
static real poly15(int k, real x, real y, real z) {
    switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return x * z;
    case 6: return y * z;
    case 7: return x * x - y * y;
    case 8: return x * x + y * y - 2 * z * z;
    case 9: return x * x + y * y + z * z;
    case 10: return x * y * y;
    case 11: return x * x * y;
    case 12: return x * x * z;
    case 13: return x * y * z;
    case 14: return x * x * y * y;
    }
    return 0;
}

static real poly7(int k, real x, real y, real z) {
    switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x - y * y;
    case 5: return x * x + y * y - 2 * z * z;
    case 6: return x * x + y * y + z * z;
    }
    return 0;
}

typedef real (*poly_fn)(int, real, real, real);

typedef struct {
    int q;
    const int (*e)[3];
    poly_fn poly;
} lattice;

static const lattice LAT15 = {15, E15, poly15};
static const lattice LAT7 = {7, E7, poly7};

static int opposite(const lattice* L, int a) {
    for (int b = 0; b < L->q; ++b)
        if (L->e[b][0] == -L->e[a][0] && L->e[b][1] == -L->e[a][1] &&
            L->e[b][2] == -L->e[a][2])
            return b;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Linear algebra: Gaussian elimination with partial pivoting (n <= 15).      */
/* ------------------------------------------------------------------------ */
static void solve(int n, real A[QMAX][QMAX], real* b, real* x) {
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabsl((long double)A[r][col]) > fabsl((long double)A[piv][col])) piv = r;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                real t = A[col][c];
                A[col][c] = A[piv][c];
                A[piv][c] = t;
            }
            real t = b[col];
            b[col] = b[piv];
            b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            real m = A[r][col] / A[col][col];
            if (m == 0) continue;
            for (int c = col; c < n; ++c) A[r][c] -= m * A[col][c];
            b[r] -= m * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        real s = b[r];
        for (int c = r + 1; c < n; ++c) s -= A[r][c] * x[c];
        x[r] = s / A[r][r];
    }
}

/* Central moments c_k = sum_a f_a P_k(e_a - u)  (eq. 14). */
static void central_moments(const lattice* L, const real* f, const real u[3], real* c) {
    for (int k = 0; k < L->q; ++k) {
        real s = 0;
        for (int a = 0; a < L->q; ++a)
            s += f[a] * L->poly(k, L->e[a][0] - u[0], L->e[a][1] - u[1], L->e[a][2] - u[2]);
        c[k] = s;
    }
}

/* The populations whose central moments about u are c. */
static void from_central(const lattice* L, const real* c, const real u[3], real* f) {
    real A[QMAX][QMAX], b[QMAX];
    for (int k = 0; k < L->q; ++k) {
        for (int a = 0; a < L->q; ++a)
            A[k][a] = L->poly(k, L->e[a][0] - u[0], L->e[a][1] - u[1], L->e[a][2] - u[2]);
        b[k] = c[k];
    }
    solve(L->q, A, b, f);
}

/* The paper's orthogonal basis vectors K_k evaluated at a particle velocity
 * e: D3Q15 (Sec. 2.2, Gram-Schmidt of the monomial set) and D3Q7
 * (Appendix C).  Used only to build the scalar source S from its printed
 * projections m^s_k = <K_k|S>. */
static real kbasis15(int k, int x, int y, int z) {
    const real e2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return x * z;
    case 6: return y * z;
    case 7: return x * x - y * y;
    case 8: return e2 - 3 * z * z;
    case 9: return e2 - 2;
    case 10: return 5 * x * e2 - 13 * x;
    case 11: return 5 * y * e2 - 13 * y;
    case 12: return 5 * z * e2 - 13 * z;
    case 13: return x * y * z;
    case 14: return 30 * (x * x * y * y + x * x * z * z + y * y * z * z) - 40 * e2 + 32;
    }
    return 0;
}

static real kbasis7(int k, int x, int y, int z) {
    switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x - y * y;
    case 5: return 2 * (x * x - z * z) - (x * x - y * y);
    case 6: return 7 * (x * x + y * y + z * z) - 6;
    }
    return 0;
}

/* Scalar source populations S^phi for a local source R at velocity u.
 * The paper prescribes the source's continuous central moments (R; 0; ...)
 * (eq. 16), turns them into raw moments by the binomial theorem, projects
 * them on the orthogonal basis (eq. 19 for D3Q15, Appendix C for D3Q7) and
 * inverts, S = K^-1 m^s (Appendix B, C).  The projections are taken as
 * printed; reading: on D3Q7 the last one is (7 (ux^2+uy^2+uz^2) - 6) R (the
 * Gram-Schmidt vector K6 weights the three squares alike; the printed 7 on
 * ux^2 alone is a typo).  On D3Q15 the printed m^s_10..12 carry continuous
 * cubes u_x^3 R although e_x^3 = e_x on the lattice, so S's lattice third-
 * and fourth-order central moments are not zero (reading: kept as printed).
 * The inverse is taken by a dense solve with the basis vectors, not with the
 * printed inverse tables. */
static void scalar_source(const lattice* L, real R, const real u[3], real* S) {
    const real ux = u[0], uy = u[1], uz = u[2];
    const real q2 = ux * ux + uy * uy + uz * uz;
    real m[QMAX], A[QMAX][QMAX];
    if (L->q == 15) {
        m[0] = R;
        m[1] = ux * R;
        m[2] = uy * R;
        m[3] = uz * R;
        m[4] = ux * uy * R;
        m[5] = ux * uz * R;
        m[6] = uy * uz * R;
        m[7] = (ux * ux - uy * uy) * R;
        m[8] = (ux * ux + uy * uy - 2 * uz * uz) * R;
        m[9] = (q2 - 2) * R;
        m[10] = 5 * (ux * ux * ux + ux * uy * uy + ux * uz * uz) * R - 13 * ux * R;
        m[11] = 5 * (ux * ux * uy + uy * uy * uy + uy * uz * uz) * R - 13 * uy * R;
        m[12] = 5 * (ux * ux * uz + uy * uy * uz + uz * uz * uz) * R - 13 * uz * R;
        m[13] = ux * uy * uz * R;
        m[14] = 30 * (ux * ux * uy * uy + ux * ux * uz * uz + uy * uy * uz * uz) * R - 40 * q2 * R +
                32 * R;
    } else {
        m[0] = R;
        m[1] = ux * R;
        m[2] = uy * R;
        m[3] = uz * R;
        m[4] = (ux * ux - uy * uy) * R;
        m[5] = (ux * ux + uy * uy - 2 * uz * uz) * R;
        m[6] = (7 * q2 - 6) * R;
    }
    for (int k = 0; k < L->q; ++k)
        for (int a = 0; a < L->q; ++a)
            A[k][a] = L->q == 15 ? kbasis15(k, L->e[a][0], L->e[a][1], L->e[a][2])
                                 : kbasis7(k, L->e[a][0], L->e[a][1], L->e[a][2]);
    solve(L->q, A, m, S);
}

/* ------------------------------------------------------------------------ */
/* Collision kernels                                                          */
/* ------------------------------------------------------------------------ */

/* Flow: cascaded central-moment collision with a body force, eq. (2a) with
 * the kernel of Appendix A (c_s^2 = 1/3).
 *
 *   rho = sum fbar,  rho u = sum fbar e + F/2                      (eq. 3)
 *   S   = the source populations (reading: the paper defers S to its
 *         earlier flow paper; here S carries the force in its first-order
 *         central moments only, i.e. central moments (0; F; 0 ... 0), the
 *         same rule Sec. 2.2 applies to the scalar source R)
 *   eta = fbar + S
 *   orders 0 and 1 of eta are kept (collision invariants: g0..g3 = 0);
 *   second order relaxes with omega[4..9] toward (0,0,0, 0,0, 3 c_s^2 rho);
 *   third order relaxes with omega[10..13] toward 0;
 *   fourth order relaxes with omega[14] toward kxx~ kyy~ / rho, where kxx~,
 *   kyy~ are the post-collision second-order central moments (reading: the
 *   paper prints the product of the post-collision moments without 1/rho;
 *   the 1/rho keeps a fluid at rest with rho != 1 a fixed point and is
 *   identical at rho = 1).  With fourth_maxwell set, the fourth-order
 *   equilibrium is instead the Maxwellian's c_s^4 rho (the value Sec. 2.2
 *   uses for the scalar); this option widens the linear stability range.
 *   post-collision = populations whose central moments are the relaxed ones.
 */
static void collide_flow(const real fbar[QF], const real F[3], const real omega[QF],
                         int fourth_maxwell, real out[QF], real* rho_out, real u_out[3]) {
    const lattice* L = &LAT15;
    real rho = 0, j[3] = {0, 0, 0};
    for (int a = 0; a < QF; ++a) {
        rho += fbar[a];
        for (int d = 0; d < 3; ++d) j[d] += fbar[a] * L->e[a][d];
    }
    real u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + F[d] / 2) / rho;

    real s_central[QF], S[QF];
    memset(s_central, 0, sizeof s_central);
    s_central[1] = F[0];
    s_central[2] = F[1];
    s_central[3] = F[2];
    from_central(L, s_central, u, S);

    real eta[QF], c[QF], ct[QF];
    for (int a = 0; a < QF; ++a) eta[a] = fbar[a] + S[a];
    central_moments(L, eta, u, c);

    real ceq2[QF];
    memset(ceq2, 0, sizeof ceq2);
    ceq2[9] = rho; /* 3 c_s^2 rho with c_s^2 = 1/3 */
    for (int k = 0; k < 4; ++k) ct[k] = c[k];
    for (int k = 4; k <= 9; ++k) ct[k] = c[k] + omega[k] * (ceq2[k] - c[k]);
    /* individual diagonal moments from the relaxed functionals 7, 8, 9 */
    real kxx = (3 * ct[7] + ct[8] + 2 * ct[9]) / 6;
    real kyy = (-3 * ct[7] + ct[8] + 2 * ct[9]) / 6;
    for (int k = 10; k <= 13; ++k) ct[k] = c[k] + omega[k] * (0 - c[k]);
    real eq14 = fourth_maxwell ? rho / 9 : kxx * kyy / rho;
    ct[14] = c[14] + omega[14] * (eq14 - c[14]);

    from_central(L, ct, u, out);
    if (rho_out) *rho_out = rho;
    if (u_out)
        for (int d = 0; d < 3; ++d) u_out[d] = u[d];
}

/* Thermal: cascaded central-moment collision for the convection-diffusion
 * equation with a local source R (eq. 13a), D3Q15 kernel of Sec. 2.2 or
 * D3Q7 kernel of Appendix C.  gbar = g - S^phi/2 is the transformed
 * distribution of eq. (13) (gbar = g when R = 0).
 *   phi = sum gbar + R/2                                             (eq. 25)
 *   eta = gbar + S^phi: the central moments of eta are those the kernel
 *     relaxes (eq. 21 uses the raw moments of gbar plus those of S^phi,
 *     reading: the lattice sums of the S^phi above);
 *   the zeroth central moment is kept (sum of the post-collision state =
 *     sum gbar + R);
 *   every other central moment k relaxes with omega[k] toward the discrete
 *   central moments of the scalar Maxwellian at phi (eq. 15):
 *     first order 0, second order xx=yy=zz=cs2 phi (so the trace is
 *     3 cs2 phi), mixed second and all third order 0, xxyy = cs2^2 phi. */
static void collide_thermal(const lattice* L, const real* gbar, const real u[3], real cs2,
                            const real* omega, real R, real* out, real* phi_out) {
    real phi = 0;
    for (int a = 0; a < L->q; ++a) phi += gbar[a];
    phi += R / 2;
    real S[QMAX], eta[QMAX], c[QMAX], ceq[QMAX], ct[QMAX];
    scalar_source(L, R, u, S);
    for (int a = 0; a < L->q; ++a) eta[a] = gbar[a] + S[a];
    central_moments(L, eta, u, c);
    memset(ceq, 0, sizeof ceq);
    ceq[0] = phi;
    if (L->q == 15) {
        ceq[9] = 3 * cs2 * phi;
        ceq[14] = cs2 * cs2 * phi;
    } else {
        ceq[6] = 3 * cs2 * phi;
    }
    ct[0] = c[0];
    for (int k = 1; k < L->q; ++k) ct[k] = c[k] + omega[k] * (ceq[k] - c[k]);
    from_central(L, ct, u, out);
    if (phi_out) *phi_out = phi;
}

/* Equilibrium populations: flow at (rho, u) (central moments rho; 0; second
 * order rho/3 on the diagonal; third order 0; xxyy = (rho/3)^2/rho) and the
 * scalar at (phi, u) (eq. 15). */
static void flow_equilibrium(real rho, const real u[3], real out[QF]) {
    real c[QF];
    memset(c, 0, sizeof c);
    c[0] = rho;
    c[9] = rho;
    c[14] = rho / 9;
    from_central(&LAT15, c, u, out);
}

static void thermal_equilibrium(const lattice* L, real phi, const real u[3], real cs2, real* out) {
    real c[QMAX];
    memset(c, 0, sizeof c);
    c[0] = phi;
    if (L->q == 15) {
        c[9] = 3 * cs2 * phi;
        c[14] = cs2 * cs2 * phi;
    } else {
        c[6] = 3 * cs2 * phi;
    }
    from_central(L, c, u, out);
}

/* ------------------------------------------------------------------------ */
/* Problem description                                                        */
/* ------------------------------------------------------------------------ */

/* Lattice-unit parameters of one run.  Layout shared with the Python wrapper
 * of this oracle (oracle.py); independent of the GPU library's own struct. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t qt;            /* thermal lattice: 7 or 15 */
    int32_t periodic;      /* bit 0/1/2: periodic in x/y/z instead of walls */
    int32_t specular;      /* scalar on the adiabatic faces: 0 bounce-back,
                              1 specular reflection */
    double omega_nu;       /* shear rates omega_4..omega_8 */
    double omega_bulk;     /* trace (bulk) rate omega_9; <= 0 means omega_nu */
    double omega_hi;       /* higher-order flow rates (omega_10..omega_14) */
    double omega_T;        /* first-order thermal rate (omega_1..omega_3) */
    double omega_hiT;      /* higher-order thermal rates */
    double cs2T;           /* c_s,phi^2 */
    double gbeta;          /* g beta of the Boussinesq force */
    double T_hot, T_cold;  /* Dirichlet walls at x = -1/2 and x = nx - 1/2 */
    double T_ref;          /* T0 of the Boussinesq force */
    int32_t fourth_maxwell; /* 4th-order flow equilibrium: 0 kxx~kyy~/rho, 1 rho/9 */
    int32_t pad2_;
    double R;              /* uniform scalar source per cell and step (eq. 4) */
} oracle_params;

/* Rest equilibrium of the scalar per unit phi: the anti-bounce-back weights. */
static void thermal_rest_weights(const oracle_params* p, real* wT) {
    real zero[3] = {0, 0, 0};
    thermal_equilibrium(p->qt == 15 ? &LAT15 : &LAT7, 1, zero, p->cs2T, wT);
}

static int nbr_index(int dx, int dy, int dz) { return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); }

/* One lattice update of one cell (collide at x after pulling eq. 2b / 13b).
 *
 * nb[27][15 + qt]: post-collision populations of the previous step in the
 * 3x3x3 neighbourhood of the cell, flow first then thermal, index
 * (dz+1)*9 + (dy+1)*3 + (dx+1).  Entries outside the domain are not read.
 *
 * Pull streaming: population a at x comes from x - e_a.  When x - e_a lies
 * outside the cavity (walls sit half a link outside the first and last
 * cells):
 *   flow:     half-way bounce-back, fbar_a(x) = F_opp(a)(x)  (no slip);
 *   thermal across an x wall: anti-bounce-back
 *             gbar_a(x) = -G_opp(a)(x) + 2 w_a T_wall (Dirichlet);
 *   thermal across only a y or z wall: bounce-back gbar_a(x) = G_opp(a)(x)
 *             (reading: zero normal flux per link for the adiabatic faces);
 *             or, with p->specular, specular reflection: the population
 *             arrives from the mirror image of its source, i.e. it left the
 *             cell (x - e_ax, y', z') with the velocity components normal to
 *             the crossed faces reversed, where y' = y if the link crosses a
 *             y face (else y - e_ay) and likewise z'.  Each link then keeps
 *             its tangential flux and carries no normal flux, so the zero-
 *             gradient (Neumann) condition holds link by link.
 *   A link that crosses an x wall and a y/z wall at once takes the Dirichlet
 *   rule (reading).
 * wT[a] is the rest equilibrium of the scalar per unit phi.
 *
 * Outputs: post-collision populations and the pre-collision macroscopic
 * fields (rho, ux, uy, uz, T) of this step. */
static void step_cell(const real* nb, int x, int y, int z, const oracle_params* p,
                      const real* wT, real* fout, real* gout, real* mac) {
    const int qt = p->qt;
    const int stride = QF + qt;
    const lattice* LT = qt == 15 ? &LAT15 : &LAT7;
    const int n[3] = {p->nx, p->ny, p->nz};
    const int pos[3] = {x, y, z};
    const real* self = nb + nbr_index(0, 0, 0) * stride;

    real fbar[QF], gbar[QMAX];
    for (int a = 0; a < QF; ++a) {
        int inside = 1;
        for (int d = 0; d < 3; ++d) {
            int s = pos[d] - E15[a][d];
            if ((s < 0 || s >= n[d]) && !((p->periodic >> d) & 1)) inside = 0;
        }
        if (inside)
            fbar[a] = nb[nbr_index(-E15[a][0], -E15[a][1], -E15[a][2]) * stride + a];
        else
            fbar[a] = self[opposite(&LAT15, a)];
    }
    for (int a = 0; a < qt; ++a) {
        int out_x = 0, out_yz = 0;
        for (int d = 0; d < 3; ++d) {
            int s = pos[d] - LT->e[a][d];
            if ((s < 0 || s >= n[d]) && !((p->periodic >> d) & 1)) {
                if (d == 0) out_x = 1;
                else out_yz = 1;
            }
        }
        int ab = opposite(LT, a);
        if (!out_x && !out_yz) {
            gbar[a] = nb[nbr_index(-LT->e[a][0], -LT->e[a][1], -LT->e[a][2]) * stride + QF + a];
        } else if (out_x) {
            real Tw = (pos[0] - LT->e[a][0] < 0) ? p->T_hot : p->T_cold;
            gbar[a] = -self[QF + ab] + 2 * wT[a] * Tw;
        } else if (!p->specular) {
            gbar[a] = self[QF + ab];
        } else {
            /* mirror the components along the crossed faces */
            int m[3] = {LT->e[a][0], LT->e[a][1], LT->e[a][2]}, d[3];
            d[0] = -LT->e[a][0];
            for (int k = 1; k < 3; ++k) {
                int s = pos[k] - LT->e[a][k];
                int out = (s < 0 || s >= n[k]) && !((p->periodic >> k) & 1);
                if (out) m[k] = -m[k];
                d[k] = out ? 0 : -LT->e[a][k];
            }
            int b = -1;
            for (int c = 0; c < qt; ++c)
                if (LT->e[c][0] == m[0] && LT->e[c][1] == m[1] && LT->e[c][2] == m[2]) b = c;
            gbar[a] = nb[nbr_index(d[0], d[1], d[2]) * stride + QF + b];
        }
    }

    /* scalar first (T = sum gbar + R/2, eq. 25), then the Boussinesq force
     * F = g beta (T - T0) z-hat, then the flow collision, then the thermal
     * collision with the flow velocity of the same step. */
    real T = p->R / 2;
    for (int a = 0; a < qt; ++a) T += gbar[a];
    real F[3] = {0, 0, p->gbeta * (T - p->T_ref)};

    real om[QF];
    for (int k = 0; k < QF; ++k) om[k] = k <= 3 ? 0 : (k <= 8 ? p->omega_nu : p->omega_hi);
    om[9] = p->omega_bulk > 0 ? p->omega_bulk : p->omega_nu;
    real rho, u[3];
    collide_flow(fbar, F, om, p->fourth_maxwell, fout, &rho, u);

    real omT[QMAX];
    for (int k = 0; k < qt; ++k) omT[k] = k == 0 ? 0 : (k <= 3 ? p->omega_T : p->omega_hiT);
    real phi;
    collide_thermal(LT, gbar, u, p->cs2T, omT, p->R, gout, &phi);

    if (mac) {
        mac[0] = rho;
        mac[1] = u[0];
        mac[2] = u[1];
        mac[3] = u[2];
        mac[4] = phi;
    }
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (double in / double out)                             */
/* ------------------------------------------------------------------------ */

static int g_threads = 0;

int ORACLE_SYM(set_threads)(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    g_threads = omp_get_max_threads();
#else
    (void)n;
    g_threads = 1;
#endif
    return g_threads;
}

int ORACLE_SYM(real_bytes)(void) { return (int)sizeof(real); }

/* Single collisions, for checking against the paper's printed kernels. */
void ORACLE_SYM(collide_flow)(const double* fbar, const double* F, const double* omega,
                              int fourth_maxwell, double* out, double* rho_u) {
    real fb[QF], Fr[3], om[QF], o[QF], rho, u[3];
    for (int a = 0; a < QF; ++a) fb[a] = fbar[a], om[a] = omega[a];
    for (int d = 0; d < 3; ++d) Fr[d] = F[d];
    collide_flow(fb, Fr, om, fourth_maxwell, o, &rho, u);
    for (int a = 0; a < QF; ++a) out[a] = (double)o[a];
    if (rho_u) {
        rho_u[0] = (double)rho;
        for (int d = 0; d < 3; ++d) rho_u[1 + d] = (double)u[d];
    }
}

void ORACLE_SYM(collide_thermal)(int qt, const double* gbar, const double* u, double cs2,
                                 const double* omega, double R, double* out) {
    const lattice* L = qt == 15 ? &LAT15 : &LAT7;
    real g[QMAX] = {0}, ur[3] = {u[0], u[1], u[2]}, om[QMAX] = {0}, o[QMAX];
    for (int a = 0; a < qt; ++a) g[a] = gbar[a], om[a] = omega[a];
    collide_thermal(L, g, ur, cs2, om, R, o, NULL);
    for (int a = 0; a < qt; ++a) out[a] = (double)o[a];
}

/* Source populations S^phi of one cell (for checking against the printed
 * inverse tables). */
void ORACLE_SYM(scalar_source)(int qt, double R, const double* u, double* S) {
    const lattice* L = qt == 15 ? &LAT15 : &LAT7;
    real ur[3] = {u[0], u[1], u[2]}, o[QMAX];
    scalar_source(L, R, ur, o);
    for (int a = 0; a < qt; ++a) S[a] = (double)o[a];
}

void ORACLE_SYM(equilibrium)(int qt, double rho, const double* u, double phi, double cs2,
                             double* feq, double* geq) {
    real ur[3] = {u[0], u[1], u[2]}, f[QF], g[QMAX];
    const lattice* L = qt == 15 ? &LAT15 : &LAT7;
    if (feq) {
        flow_equilibrium(rho, ur, f);
        for (int a = 0; a < QF; ++a) feq[a] = (double)f[a];
    }
    if (geq) {
        thermal_equilibrium(L, phi, ur, cs2, g);
        for (int a = 0; a < qt; ++a) geq[a] = (double)g[a];
    }
}

/* State layout: F[a][z][y][x] (15 arrays), G[a][z][y][x] (qt arrays). */
static size_t cell_of(const oracle_params* p, int x, int y, int z) {
    return ((size_t)z * p->ny + y) * p->nx + x;
}

static void gather_nb(const oracle_params* p, const real* F, const real* G, size_t ncell, int x,
                      int y, int z, real* nb) {
    const int stride = QF + p->qt;
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int s[3] = {x + dx, y + dy, z + dz}, ok = 1;
                for (int d = 0; d < 3; ++d)
                    if (s[d] < 0 || s[d] >= n[d]) {
                        if ((p->periodic >> d) & 1) s[d] = (s[d] + n[d]) % n[d];
                        else ok = 0;
                    }
                real* dst = nb + nbr_index(dx, dy, dz) * stride;
                if (!ok) {
                    for (int a = 0; a < stride; ++a) dst[a] = NAN;
                    continue;
                }
                size_t c = cell_of(p, s[0], s[1], s[2]);
                for (int a = 0; a < QF; ++a) dst[a] = F[a * ncell + c];
                for (int a = 0; a < p->qt; ++a) dst[QF + a] = G[a * ncell + c];
            }
}

/* Advance nsteps.  F, G hold the post-collision state (double) on entry and
 * on exit; mac (optional, [5][ncell]) receives rho, ux, uy, uz, T of the last
 * step (pre-collision moments of that step). */
int ORACLE_SYM(run)(const oracle_params* p, int64_t nsteps, double* F, double* G, double* mac) {
    const size_t ncell = (size_t)p->nx * p->ny * p->nz;
    const int qt = p->qt;
    if (qt != 7 && qt != 15) return -1;
    real* A = (real*)malloc(sizeof(real) * ncell * (QF + qt));
    real* B = (real*)malloc(sizeof(real) * ncell * (QF + qt));
    if (!A || !B) {
        free(A);
        free(B);
        return -2;
    }
    for (size_t i = 0; i < ncell * QF; ++i) A[i] = F[i];
    for (size_t i = 0; i < ncell * qt; ++i) A[ncell * QF + i] = G[i];
    real wT[QMAX];
    thermal_rest_weights(p, wT);
    for (int64_t s = 0; s < nsteps; ++s) {
        const real* Fi = A;
        const real* Gi = A + ncell * QF;
        real* Fo = B;
        real* Go = B + ncell * QF;
        const int last = (s == nsteps - 1);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < p->nz; ++z) {
            real nb[27 * (QF + QMAX)], fo[QF], go[QMAX], m[5];
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    gather_nb(p, Fi, Gi, ncell, x, y, z, nb);
                    step_cell(nb, x, y, z, p, wT, fo, go, m);
                    size_t c = cell_of(p, x, y, z);
                    for (int a = 0; a < QF; ++a) Fo[a * ncell + c] = fo[a];
                    for (int a = 0; a < qt; ++a) Go[a * ncell + c] = go[a];
                    if (last && mac)
                        for (int k = 0; k < 5; ++k) mac[k * ncell + c] = (double)m[k];
                }
        }
        real* t = A;
        A = B;
        B = t;
    }
    for (size_t i = 0; i < ncell * QF; ++i) F[i] = (double)A[i];
    for (size_t i = 0; i < ncell * qt; ++i) G[i] = (double)A[ncell * QF + i];
    free(A);
    free(B);
    return 0;
}

/* One update of selected cells from their neighbourhoods.
 * nb: [n][27][15+qt] post-collision populations of the previous step (see
 * step_cell); pos: [n][3] cell coordinates; fout [n][15], gout [n][qt],
 * mac [n][5]. */
void ORACLE_SYM(step_cells)(const oracle_params* p, int64_t n, const double* nb,
                            const int32_t* pos, double* fout, double* gout, double* mac) {
    const int stride = QF + p->qt;
    real wT[QMAX];
    thermal_rest_weights(p, wT);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        real b[27 * (QF + QMAX)], fo[QF], go[QMAX], m[5];
        for (int k = 0; k < 27 * stride; ++k) b[k] = nb[i * 27 * stride + k];
        step_cell(b, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], p, wT, fo, go, m);
        for (int a = 0; a < QF; ++a) fout[i * QF + a] = (double)fo[a];
        for (int a = 0; a < p->qt; ++a) gout[i * p->qt + a] = (double)go[a];
        if (mac)
            for (int k = 0; k < 5; ++k) mac[i * 5 + k] = (double)m[k];
    }
}

/* Equilibrium state from macroscopic fields ([ncell] each, rho may be NULL
 * for rho = 1).  The scalar populations are the equilibrium at T - R/2, so
 * that the first step sees T (eq. 25 with the source). */
void ORACLE_SYM(init_equilibrium)(const oracle_params* p, const double* rho, const double* ux,
                                  const double* uy, const double* uz, const double* T, double* F,
                                  double* G) {
    const size_t ncell = (size_t)p->nx * p->ny * p->nz;
    const lattice* LT = p->qt == 15 ? &LAT15 : &LAT7;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < (int64_t)ncell; ++c) {
        real u[3] = {ux ? ux[c] : 0, uy ? uy[c] : 0, uz ? uz[c] : 0}, f[QF], g[QMAX];
        flow_equilibrium(rho ? rho[c] : 1, u, f);
        thermal_equilibrium(LT, (T ? T[c] : 0) - p->R / 2, u, p->cs2T, g);
        for (int a = 0; a < QF; ++a) F[a * ncell + c] = (double)f[a];
        for (int a = 0; a < p->qt; ++a) G[a * ncell + c] = (double)g[a];
    }
}

/* Local Nusselt numbers on the two Dirichlet walls, from the stored
 * post-collision thermal populations G.
 *
 * The heat that crosses the hot wall (x = -1/2) into the first fluid layer
 * per step is, per link, what anti-bounce-back returns minus what left:
 *   gbar_a - G_opp(a) = 2 (w_a T_hot - G_opp(a)),  for links with e_ax > 0.
 * The cold wall (x = nx - 1/2) likewise takes out 2 (G_a - w_a T_cold) per
 * link with e_ax > 0.  Nu = q L / (alpha dT) with L = nx, dT = T_hot -
 * T_cold, alpha the thermal diffusivity (eq. 23).  Reading: the paper prints
 * Nu as the wall-normal temperature gradient integrated over the wall; the
 * link flux is the lattice's exact form of that gradient (Nu = 1 for pure
 * conduction).
 * nu_hot, nu_cold: [nz][ny]. */
void ORACLE_SYM(nusselt)(const oracle_params* p, const double* G, double alpha, double* nu_hot,
                         double* nu_cold) {
    const size_t ncell = (size_t)p->nx * p->ny * p->nz;
    const lattice* LT = p->qt == 15 ? &LAT15 : &LAT7;
    real wT[QMAX];
    thermal_rest_weights(p, wT);
    const real dT = p->T_hot - p->T_cold;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y) {
            real qh = 0, qc = 0;
            for (int a = 0; a < LT->q; ++a) {
                if (LT->e[a][0] <= 0) continue;
                int ab = opposite(LT, a);
                qh += 2 * (wT[a] * p->T_hot - G[ab * ncell + cell_of(p, 0, y, z)]);
                qc += 2 * (G[a * ncell + cell_of(p, p->nx - 1, y, z)] - wT[a] * p->T_cold);
            }
            nu_hot[(size_t)z * p->ny + y] = (double)(qh * p->nx / (alpha * dT));
            nu_cold[(size_t)z * p->ny + y] = (double)(qc * p->nx / (alpha * dT));
        }
}
