/*
 * FP64 CPU oracle for the D3Q19 cascaded (central-moment, multiple-relaxation-
 * time) lattice Boltzmann method for power-law fluids of Adam, Hajabdollahi and
 * Premnath, "Cascaded lattice Boltzmann modeling and simulations of three-
 * dimensional non-Newtonian fluid flows" (arXiv:1908.05396).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, table
 * or header with the GPU library.
 *
 * What it computes, per time step (Sec. 3):
 *   1. rho = sum f, rho u = sum e f                              (Eq. hydrodynamic fields)
 *   2. optional body force: half of the source added before and after
 *      collision (symmetrized operator splitting; Sec. 3 intro and Sec. 4.2
 *      defer the scheme to an external reference, the reading used here is:
 *      the source has central moments (0, F, 0, ..., 0) about the velocity
 *      u = (sum e f + F/2)/rho, both halves use that u)
 *   3. central moments kappa = <(e-u)^mnp | f> by direct summation
 *      (discrete central-moment definitions, Sec. 3)
 *   4. local relaxation rate omega^nu of the second-order moments from the
 *      power-law apparent viscosity (Eqs. 4-6, Eq. local variations of
 *      relaxation times, Eq. strain rate tensor).  The strain rate depends on
 *      omega^nu itself; the oracle solves that local equation exactly by
 *      bisection.  The kinematic viscosity is clipped to [nu_min, nu_max].
 *   5. relaxation of each central-moment combination to its (factorized)
 *      attractor: Eq. central moment relaxation with the attractors of
 *      Eq. discrete central moment attractors.  The fourth-order attractors
 *      are products of post-collision second-order central moments divided
 *      by rho, the factorization of the density-normalized distribution:
 *      at equilibrium this gives c_s^4 rho, the Maxwellian value listed in
 *      Sec. 3.  The paper prints the product without 1/rho; that form is
 *      available with attractor_literal = 1, but it makes the scheme
 *      linearly unstable to density perturbations (equal at rho = 1).
 *   6. post-collision populations f~ = f + Omega (Eq. cascaded collision):
 *      Omega is the unique population change whose central moments equal
 *      the relaxed minus the incoming ones (linear solve with the per-node
 *      moment matrix)
 *   7. streaming f(x + e, t+1) = f~(x, t) (Eq. cascaded streaming) with
 *      periodic axes, half-way bounce-back walls and a moving-lid momentum
 *      correction (Sec. 4.1, 4.2, 4.3).
 *
 * model = 1 selects instead the single-relaxation-time (BGK) comparison model
 * of Sec. 5 with the same power-law relaxation time (see collide_node_srt).
 *
 * Conventions: lattice units, c_s^2 = 1/3, node index x + nx*(y + ny*z),
 * populations stored as structure of arrays f[alpha*N + node].
 * No fast-math: every operation is IEEE double with round-to-nearest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define CS2 (1.0 / 3.0)

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic[3];   /* 1 = periodic axis, 0 = bounce-back walls at both ends */
    int32_t lid_face;      /* 0 none; 1 -x, 2 +x, 3 -y, 4 +y, 5 -z, 6 +z */
    int32_t attractor_literal; /* 1: fourth-order attractors without 1/rho (see below) */
    double K;              /* consistency coefficient mu_p (Eq. 5) */
    double n;              /* power-law index (Eq. 5) */
    double nu_min, nu_max; /* clip of the apparent kinematic viscosity */
    double omega_bulk;     /* omega_9 (the paper sets it to 1) */
    double omega_high[9];  /* omega_10 ... omega_18 (the paper sets them to 1) */
    double force[3];       /* body force per unit volume */
    double lid_velocity[3];
    double rho_wall;       /* density in the moving-wall correction */
    int32_t model;         /* 0: the cascaded scheme; 1: single-relaxation-time BGK (comparison model) */
    int32_t pad_;
    const uint8_t *flags;  /* per-node solid flags (NULL: every node is fluid): 0 fluid, 1 wall,
                              2 wall moving with lid_velocity */
} orc_params;

enum { FLAG_FLUID = 0, FLAG_WALL = 1, FLAG_MOVING_WALL = 2 };

static int is_solid(const orc_params *p, int64_t i) { return p->flags && p->flags[i] != FLAG_FLUID; }

/* D3Q19 particle velocities, alpha = 0..18, read off the component vectors
 * |e_x>, |e_y>, |e_z> given with the moment basis in Sec. 3. */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

/* The 19 independent central moments supported by D3Q19, as exponents
 * (m, n, p) of (e_x - u_x)^m (e_y - u_y)^n (e_z - u_z)^p. */
enum {
    M_0, M_X, M_Y, M_Z, M_XY, M_XZ, M_YZ, M_XX, M_YY, M_ZZ,
    M_XYY, M_XZZ, M_XXY, M_YZZ, M_XXZ, M_YYZ, M_XXYY, M_XXZZ, M_YYZZ
};
static const int MEXP[Q][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
    {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 1, 2},
    {2, 0, 1}, {0, 2, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};

/* Combinations Phi_j of the central moments that relax with omega_j, one per
 * basis vector K_j of the orthogonal collision matrix (Sec. 3):
 * K_4..K_6 -> xy, xz, yz; K_7 -> xx-yy; K_8 -> xx+yy-2zz; K_9 -> xx+yy+zz;
 * K_10..K_12 -> xyy+xzz, xxy+yzz, xxz+yyz; K_13..K_15 -> xyy-xzz, yzz-xxy,
 * xxz-yyz; K_16..K_18 -> xxyy+xxzz+yyzz, xxyy+xxzz-2yyzz, xxyy-xxzz.
 * Rows 0..3 are the conserved moments themselves. */
static double CMB[Q][Q];
static double CMB_INV[Q][Q];
static int OPP[Q];
static double W[Q];
static int tables_ready = 0;

static double ipow(double b, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

/* Solve A x = b (n x n, row-major, A and b are overwritten) by Gaussian
 * elimination with partial pivoting.  Returns 0 on success. */
static int solve_linear(int nn, double *A, double *b, double *x) {
    for (int c = 0; c < nn; ++c) {
        int piv = c;
        double best = fabs(A[c * nn + c]);
        for (int r = c + 1; r < nn; ++r) {
            double v = fabs(A[r * nn + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < nn; ++k) {
                double t = A[c * nn + k]; A[c * nn + k] = A[piv * nn + k]; A[piv * nn + k] = t;
            }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < nn; ++r) {
            double fct = A[r * nn + c] / A[c * nn + c];
            if (fct == 0.0) continue;
            for (int k = c; k < nn; ++k) A[r * nn + k] -= fct * A[c * nn + k];
            b[r] -= fct * b[c];
        }
    }
    for (int r = nn - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < nn; ++k) s -= A[r * nn + k] * x[k];
        x[r] = s / A[r * nn + r];
    }
    return 0;
}

/* Moment matrix about velocity u: row k holds the k-th central monomial
 * evaluated at each particle velocity, so that kappa = M f. */
static void moment_matrix(const double u[3], double M[Q * Q]) {
    for (int k = 0; k < Q; ++k)
        for (int a = 0; a < Q; ++a)
            M[k * Q + a] = ipow(EX[a] - u[0], MEXP[k][0]) *
                           ipow(EY[a] - u[1], MEXP[k][1]) *
                           ipow(EZ[a] - u[2], MEXP[k][2]);
}

static void matvec(const double M[Q * Q], const double *v, double *out) {
    for (int k = 0; k < Q; ++k) {
        double s = 0.0;
        for (int a = 0; a < Q; ++a) s += M[k * Q + a] * v[a];
        out[k] = s;
    }
}

/* f = M(u)^{-1} kappa */
static int populations_from_central(const double u[3], const double kappa[Q], double f[Q]) {
    double M[Q * Q], b[Q];
    moment_matrix(u, M);
    memcpy(b, kappa, sizeof(b));
    return solve_linear(Q, M, b, f);
}

static void init_tables(void) {
    if (tables_ready) return;
    memset(CMB, 0, sizeof(CMB));
    CMB[0][M_0] = 1; CMB[1][M_X] = 1; CMB[2][M_Y] = 1; CMB[3][M_Z] = 1;
    CMB[4][M_XY] = 1; CMB[5][M_XZ] = 1; CMB[6][M_YZ] = 1;
    CMB[7][M_XX] = 1; CMB[7][M_YY] = -1;
    CMB[8][M_XX] = 1; CMB[8][M_YY] = 1; CMB[8][M_ZZ] = -2;
    CMB[9][M_XX] = 1; CMB[9][M_YY] = 1; CMB[9][M_ZZ] = 1;
    CMB[10][M_XYY] = 1; CMB[10][M_XZZ] = 1;
    CMB[11][M_XXY] = 1; CMB[11][M_YZZ] = 1;
    CMB[12][M_XXZ] = 1; CMB[12][M_YYZ] = 1;
    CMB[13][M_XYY] = 1; CMB[13][M_XZZ] = -1;
    CMB[14][M_YZZ] = 1; CMB[14][M_XXY] = -1;
    CMB[15][M_XXZ] = 1; CMB[15][M_YYZ] = -1;
    CMB[16][M_XXYY] = 1; CMB[16][M_XXZZ] = 1; CMB[16][M_YYZZ] = 1;
    CMB[17][M_XXYY] = 1; CMB[17][M_XXZZ] = 1; CMB[17][M_YYZZ] = -2;
    CMB[18][M_XXYY] = 1; CMB[18][M_XXZZ] = -1;
    /* inverse of the combination matrix, column by column */
    for (int c = 0; c < Q; ++c) {
        double A[Q * Q], b[Q], x[Q];
        for (int r = 0; r < Q; ++r) {
            for (int k = 0; k < Q; ++k) A[r * Q + k] = CMB[r][k];
            b[r] = (r == c) ? 1.0 : 0.0;
        }
        solve_linear(Q, A, b, x);
        for (int r = 0; r < Q; ++r) CMB_INV[r][c] = x[r];
    }
    for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b)
            if (EX[b] == -EX[a] && EY[b] == -EY[a] && EZ[b] == -EZ[a]) OPP[a] = b;
    /* Weights: the rest state (rho = 1, u = 0) of the attractors: second-order
     * diagonal central moments c_s^2 rho, fourth-order ones their products,
     * every other non-conserved moment zero. */
    {
        double k0[Q] = {0}, u0[3] = {0, 0, 0};
        k0[M_0] = 1.0;
        k0[M_XX] = k0[M_YY] = k0[M_ZZ] = CS2;
        k0[M_XXYY] = k0[M_XXZZ] = k0[M_YYZZ] = CS2 * CS2;
        populations_from_central(u0, k0, W);
    }
    tables_ready = 1;
}

/* ---------------------------------------------------------------------- */
/* Power-law relaxation rate (Sec. 3.2)                                     */
/* ---------------------------------------------------------------------- */

/* Shear-rate magnitude |gamma| from the strain-rate tensor obtained from the
 * non-equilibrium moments m4..m9 at a trial omega^nu (Eq. strain rate tensor,
 * Eq. shear rate expression). */
static double shear_rate(double om_nu, double om_zeta, double rho, const double m[10]) {
    double sxy = -1.5 / rho * om_nu * m[4];
    double sxz = -1.5 / rho * om_nu * m[5];
    double syz = -1.5 / rho * om_nu * m[6];
    double sxx = -0.5 / rho * (om_nu * (m[7] + m[8]) + om_zeta * m[9]);
    double syy = -0.5 / rho * (om_nu * (-2.0 * m[7] + m[8]) + om_zeta * m[9]);
    double szz = -0.5 / rho * (om_nu * (m[7] - 2.0 * m[8]) + om_zeta * m[9]);
    return sqrt(2.0 * (sxx * sxx + syy * syy + szz * szz +
                       2.0 * (sxy * sxy + syz * syz + sxz * sxz)));
}

/* Apparent kinematic viscosity mu(|gamma|)/rho of the power-law fluid
 * (Eq. 6), clipped to [nu_min, nu_max]. */
static double clipped_nu(const orc_params *p, double gamma, double rho) {
    double nu = p->K * pow(gamma, p->n - 1.0) / rho;
    if (!(nu >= p->nu_min)) nu = (nu != nu) ? nu : p->nu_min;  /* keep NaN visible */
    if (nu > p->nu_max) nu = p->nu_max;
    return nu;
}

/* Residual of the local equation tau = 1/omega^nu = mu/(rho c_s^2) + 1/2
 * (Eq. local variations of relaxation times) at a trial tau. */
static double tau_residual(const orc_params *p, double tau, double rho, const double m[10]) {
    double g = shear_rate(1.0 / tau, p->omega_bulk, rho, m);
    return tau - 0.5 - clipped_nu(p, g, rho) / CS2;
}

/* Exact local omega^nu by bisection on tau over the clip interval.  The
 * residual is negative at the lower end and positive at the upper end; the
 * loop runs until the bracket cannot be split further in double precision. */
static double solve_omega_nu(const orc_params *p, double rho, const double m[10]) {
    double lo = p->nu_min / CS2 + 0.5, hi = p->nu_max / CS2 + 0.5;
    double hlo = tau_residual(p, lo, rho, m);
    double hhi = tau_residual(p, hi, rho, m);
    if (hlo != hlo || hhi != hhi) return NAN;
    if (hlo >= 0.0) return 1.0 / lo;
    if (hhi <= 0.0) return 1.0 / hi;
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double h = tau_residual(p, mid, rho, m);
        if (h > 0.0) { hi = mid; hhi = h; }
        else { lo = mid; hlo = h; }
    }
    double tau = (fabs(hlo) <= fabs(hhi)) ? lo : hi;
    return 1.0 / tau;
}

/* ---------------------------------------------------------------------- */
/* Single-relaxation-time comparison model (Sec. 5)                         */
/* ---------------------------------------------------------------------- */
/* The paper compares its scheme with the SRT (BGK) model, in which every
 * population relaxes at the one rate 1/tau, tau set locally by the same
 * power-law equation; it does not print that model.  Textbook form used
 * here (Qian, d'Humieres & Lallemand 1992; Kruger et al. 2017, Ch. 3, 4, 10):
 *   f_eq = w rho (1 + e.u/cs2 + (e.u)^2/(2 cs2^2) - u.u/(2 cs2)),
 *   Pi_neq = sum e e (f - f_eq),  S = -Pi_neq / (2 rho cs2 tau),
 *   f~ = f - (f - f_eq) / tau.  Unforced. */
static double shear_rate_srt(double tau, double rho, const double pi[6]) {
    double c = -1.0 / (2.0 * rho * CS2 * tau);
    double sxx = c * pi[0], syy = c * pi[1], szz = c * pi[2];
    double sxy = c * pi[3], sxz = c * pi[4], syz = c * pi[5];
    return sqrt(2.0 * (sxx * sxx + syy * syy + szz * szz + 2.0 * (sxy * sxy + sxz * sxz + syz * syz)));
}

static double srt_residual(const orc_params *p, double tau, double rho, const double pi[6]) {
    return tau - 0.5 - clipped_nu(p, shear_rate_srt(tau, rho, pi), rho) / CS2;
}

/* The same bisection on tau over the clip interval as for the cascaded rate. */
static double solve_tau_srt(const orc_params *p, double rho, const double pi[6]) {
    double lo = p->nu_min / CS2 + 0.5, hi = p->nu_max / CS2 + 0.5;
    double hlo = srt_residual(p, lo, rho, pi), hhi = srt_residual(p, hi, rho, pi);
    if (hlo != hlo || hhi != hhi) return NAN;
    if (hlo >= 0.0) return lo;
    if (hhi <= 0.0) return hi;
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double h = srt_residual(p, mid, rho, pi);
        if (h > 0.0) { hi = mid; hhi = h; }
        else { lo = mid; hlo = h; }
    }
    return (fabs(hlo) <= fabs(hhi)) ? lo : hi;
}

static int collide_node_srt(const orc_params *p, const double *f, double *fout, double *omega_out) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Q; ++a) {
        rho += f[a];
        j[0] += EX[a] * f[a]; j[1] += EY[a] * f[a]; j[2] += EZ[a] * f[a];
    }
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double feq[Q], pi[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < Q; ++a) {
        double eu = EX[a] * u[0] + EY[a] * u[1] + EZ[a] * u[2];
        feq[a] = W[a] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
        double ne = f[a] - feq[a];
        pi[0] += EX[a] * EX[a] * ne; pi[1] += EY[a] * EY[a] * ne; pi[2] += EZ[a] * EZ[a] * ne;
        pi[3] += EX[a] * EY[a] * ne; pi[4] += EX[a] * EZ[a] * ne; pi[5] += EY[a] * EZ[a] * ne;
    }
    double tau = solve_tau_srt(p, rho, pi);
    for (int a = 0; a < Q; ++a) fout[a] = f[a] - (f[a] - feq[a]) / tau;
    if (omega_out) *omega_out = 1.0 / tau;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Collision of one node                                                    */
/* ---------------------------------------------------------------------- */

int orc_collide_node(const orc_params *p, const double *fin, double *fout, double *omega_out) {
    init_tables();
    if (p->model == 1) return collide_node_srt(p, fin, fout, omega_out);
    double f[Q];
    memcpy(f, fin, sizeof(f));
    const double *F = p->force;
    int forced = (F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0);

    /* density and momentum (Eq. hydrodynamic fields) */
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int a = 0; a < Q; ++a) {
        rho += f[a];
        j[0] += EX[a] * f[a];
        j[1] += EY[a] * f[a];
        j[2] += EZ[a] * f[a];
    }
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / rho;

    /* first half of the source: populations whose central moments about u
     * are (0, F, 0, ..., 0) */
    double S[Q] = {0};
    if (forced) {
        double s[Q] = {0};
        s[M_X] = F[0]; s[M_Y] = F[1]; s[M_Z] = F[2];
        if (populations_from_central(u, s, S)) return -1;
        for (int a = 0; a < Q; ++a) f[a] += 0.5 * S[a];
    }

    /* raw moments (Eq. raw moments) and central moments about u */
    double M0[Q * Q], Mu[Q * Q], zero[3] = {0, 0, 0};
    double raw[Q], kap[Q];
    moment_matrix(zero, M0);
    moment_matrix(u, Mu);
    matvec(M0, f, raw);
    matvec(Mu, f, kap);

    /* non-equilibrium second-order moments in terms of raw moments (Sec. 3.2) */
    double m[10] = {0};
    m[4] = raw[M_XY] - rho * u[0] * u[1];
    m[5] = raw[M_XZ] - rho * u[0] * u[2];
    m[6] = raw[M_YZ] - rho * u[1] * u[2];
    m[7] = (raw[M_XX] - raw[M_YY]) - rho * (u[0] * u[0] - u[1] * u[1]);
    m[8] = (raw[M_XX] - raw[M_ZZ]) - rho * (u[0] * u[0] - u[2] * u[2]);
    m[9] = (raw[M_XX] + raw[M_YY] + raw[M_ZZ]) -
           (rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + rho);

    double om_nu = solve_omega_nu(p, rho, m);
    if (omega_out) *omega_out = om_nu;

    double om[Q];
    for (int k = 0; k < Q; ++k) om[k] = 0.0;
    for (int k = 4; k <= 8; ++k) om[k] = om_nu;
    om[9] = p->omega_bulk;
    for (int k = 10; k <= 18; ++k) om[k] = p->omega_high[k - 10];

    /* combinations, relaxed toward their attractors (second order first, the
     * fourth-order attractors use the post-collision second-order moments) */
    double phi[Q], phit[Q], kt[Q];
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += CMB[r][k] * kap[k];
        phi[r] = s;
    }
    double att[Q] = {0};
    att[9] = 3.0 * CS2 * rho;            /* trace: xx + yy + zz -> 3 c_s^2 rho */
    for (int r = 0; r < Q; ++r) phit[r] = phi[r];
    for (int r = 4; r <= 15; ++r) phit[r] = phi[r] + om[r] * (att[r] - phi[r]);
    /* the first central moments of the half-forced state vanish; keep them exact */
    phit[1] = phit[2] = phit[3] = 0.0;
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += CMB_INV[r][k] * phit[k];
        kt[r] = s;
    }
    double norm = p->attractor_literal ? 1.0 : rho;
    double axxyy = kt[M_XX] * kt[M_YY] / norm;
    double axxzz = kt[M_XX] * kt[M_ZZ] / norm;
    double ayyzz = kt[M_YY] * kt[M_ZZ] / norm;
    att[16] = axxyy + axxzz + ayyzz;
    att[17] = axxyy + axxzz - 2.0 * ayyzz;
    att[18] = axxyy - axxzz;
    for (int r = 16; r <= 18; ++r) phit[r] = phi[r] + om[r] * (att[r] - phi[r]);
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += CMB_INV[r][k] * phit[k];
        kt[r] = s;
    }

    /* post-collision populations: f~ = f + Omega (Eq. cascaded collision),
     * with Omega the unique change of populations whose central moments
     * change by kappa~ - kappa.  Solving for the (small) change rather than
     * for f~ itself keeps the linear solve's rounding proportional to the
     * change. */
    double dk[Q], df[Q];
    for (int r = 0; r < Q; ++r) dk[r] = kt[r] - kap[r];
    if (populations_from_central(u, dk, df)) return -1;
    for (int a = 0; a < Q; ++a) fout[a] = f[a] + df[a];
    if (forced)
        for (int a = 0; a < Q; ++a) fout[a] += 0.5 * S[a];
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Lattice-wide operations                                                  */
/* ---------------------------------------------------------------------- */

static int64_t nnodes(const orc_params *p) {
    return (int64_t)p->nx * p->ny * p->nz;
}

static int valid_params(const orc_params *p) {
    if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return 0;
    if (!(p->K > 0.0) || !(p->n > 0.0)) return 0;
    if (!(p->nu_min > 0.0) || !(p->nu_max > p->nu_min)) return 0;
    if (p->lid_face < 0 || p->lid_face > 6) return 0;
    if (p->model != 0 && p->model != 1) return 0;
    if (p->model == 1 && (p->force[0] != 0.0 || p->force[1] != 0.0 || p->force[2] != 0.0)) return 0;
    return 1;
}

int orc_weights(double *w) {
    init_tables();
    memcpy(w, W, sizeof(W));
    return 0;
}

int orc_velocities(int32_t *e) {
    for (int a = 0; a < Q; ++a) {
        e[3 * a + 0] = EX[a];
        e[3 * a + 1] = EY[a];
        e[3 * a + 2] = EZ[a];
    }
    return 0;
}

int orc_opposite(int32_t *opp) {
    init_tables();
    for (int a = 0; a < Q; ++a) opp[a] = OPP[a];
    return 0;
}

int orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

/* Collide every fluid node: fout = C(fin); omega (nullable) receives
 * omega^nu.  Solid nodes (flags) are not part of the fluid: they hold the
 * rest populations w and report omega = 0. */
int orc_collide(const orc_params *p, const double *fin, double *fout, double *omega) {
    if (!valid_params(p)) return -1;
    init_tables();
    int64_t N = nnodes(p);
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t i = 0; i < N; ++i) {
        double a_in[Q], a_out[Q], om;
        if (is_solid(p, i)) {
            for (int a = 0; a < Q; ++a) fout[a * N + i] = W[a];
            if (omega) omega[i] = 0.0;
            continue;
        }
        for (int a = 0; a < Q; ++a) a_in[a] = fin[a * N + i];
        err |= orc_collide_node(p, a_in, a_out, &om) ? 1 : 0;
        for (int a = 0; a < Q; ++a) fout[a * N + i] = a_out[a];
        if (omega) omega[i] = om;
    }
    return err ? -2 : 0;
}

/* Is a ghost node (outside the lattice on at least one bounce-back axis) part
 * of the moving lid?  Every ghost in the lid plane moves, edges and corners
 * of that plane included. */
static int in_lid_plane(const orc_params *p, int sx, int sy, int sz) {
    switch (p->lid_face) {
    case 1: return sx == -1;
    case 2: return sx == p->nx;
    case 3: return sy == -1;
    case 4: return sy == p->ny;
    case 5: return sz == -1;
    case 6: return sz == p->nz;
    default: return 0;
    }
}

/* Streaming (Eq. cascaded streaming) in pull form: the population moving
 * along e arriving at x left x - e one step earlier.  If x - e is outside the
 * lattice across a wall, or is a node flagged solid, half-way bounce-back
 * (Sec. 4.1) returns the population that left x toward the wall, plus the
 * moving-wall momentum term 2 w rho_w (e . U_w) / c_s^2 (Sec. 4.3) when the
 * wall moves: a ghost in the lid plane, or a node flagged as moving wall.
 * Solid nodes keep the rest populations. */
int orc_stream(const orc_params *p, const double *ft, double *f) {
    if (!valid_params(p)) return -1;
    init_tables();
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    int64_t N = nnodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        if (is_solid(p, i)) {
            for (int a = 0; a < Q; ++a) f[a * N + i] = W[a];
            continue;
        }
        for (int a = 0; a < Q; ++a) {
            int sx = x - EX[a], sy = y - EY[a], sz = z - EZ[a];
            int ghost = 0;
            int wx = sx, wy = sy, wz = sz;
            if (p->periodic[0]) wx = (sx + nx) % nx; else if (sx < 0 || sx >= nx) ghost = 1;
            if (p->periodic[1]) wy = (sy + ny) % ny; else if (sy < 0 || sy >= ny) ghost = 1;
            if (p->periodic[2]) wz = (sz + nz) % nz; else if (sz < 0 || sz >= nz) ghost = 1;
            int moving = 0;
            if (!ghost) {
                int64_t s = (int64_t)wx + (int64_t)nx * ((int64_t)wy + (int64_t)ny * wz);
                if (!is_solid(p, s)) {
                    f[a * N + i] = ft[a * N + s];
                    continue;
                }
                moving = p->flags[s] == FLAG_MOVING_WALL;
            } else {
                moving = in_lid_plane(p, sx, sy, sz);
            }
            {
                double corr = 0.0;
                if (moving) {
                    double eu = EX[a] * p->lid_velocity[0] + EY[a] * p->lid_velocity[1] +
                                EZ[a] * p->lid_velocity[2];
                    corr = 2.0 * W[a] * p->rho_wall * eu / CS2;
                }
                f[a * N + i] = ft[OPP[a] * N + i] + corr;
            }
        }
    }
    return 0;
}

/* Advance the pre-collision state f by `steps` collide + stream steps. */
int orc_run(const orc_params *p, double *f, int64_t steps) {
    if (!valid_params(p)) return -1;
    int64_t N = nnodes(p);
    double *ft = (double *)malloc(sizeof(double) * Q * N);
    if (!ft) return -3;
    int err = 0;
    for (int64_t t = 0; t < steps && !err; ++t) {
        err = orc_collide(p, f, ft, NULL);
        if (!err) err = orc_stream(p, ft, f);
    }
    free(ft);
    return err;
}

/* Density and velocity of a pre-collision state: rho = sum f and
 * u = (sum e f + F/2) / rho.  u is stored as three planes (ux, uy, uz).
 * Solid nodes report rho = 1, u = 0. */
int orc_macroscopic(const orc_params *p, const double *f, double *rho, double *u) {
    if (!valid_params(p)) return -1;
    int64_t N = nnodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if (is_solid(p, i)) {
            rho[i] = 1.0;
            u[i] = u[N + i] = u[2 * N + i] = 0.0;
            continue;
        }
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int a = 0; a < Q; ++a) {
            double v = f[a * N + i];
            r += v; jx += EX[a] * v; jy += EY[a] * v; jz += EZ[a] * v;
        }
        rho[i] = r;
        u[i] = (jx + 0.5 * p->force[0]) / r;
        u[N + i] = (jy + 0.5 * p->force[1]) / r;
        u[2 * N + i] = (jz + 0.5 * p->force[2]) / r;
    }
    return 0;
}
