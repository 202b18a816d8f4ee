/*
 * Plain FP64 CPU oracle: D2Q9 pseudopotential MRT lattice Boltzmann step with
 * the surface-tension source term of Li & Luo (arXiv:1306.6445).
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).  Written to be read against the
 * paper, not to be fast: the moment transform is a dense 9x9 product with a
 * matrix built from the moment polynomials and inverted by Gauss-Jordan
 * elimination, streaming uses two arrays, and every quantity is formed in the
 * order the paper states it:
 *   density (Eq. 6) -> psi (Section II; Eq. 23) -> force F (Eq. 7) and
 *   source tensor Q (Eq. 19) -> velocity (Eq. 6) -> m = M f, m_eq (Eq. 3),
 *   S (Eqs. 5, 8), C (Eq. 18) -> m* (Eq. 17) -> f* = M^-1 m* -> streaming (Eq. 4).
 * The OpenMP pragma only splits the node loop across threads; every node's
 * arithmetic is the same whatever the thread count.
 *
 * Readings where the paper is silent (stated again where they are used):
 *  - M is the orthogonal D2Q9 basis whose equilibrium moments are exactly
 *    Eq. (3) and whose forcing moments are exactly Eq. (5); lattice units
 *    c = dt = 1, cs^2 = 1/3.
 *  - Walls are halfway bounce-back; at a wall the psi of the missing neighbour
 *    row/column is the psi of the adjacent fluid node (neutral wetting).
 *  - The Carnahan-Starling EOS is p = rho R T (1+eta+eta^2-eta^3)/(1-eta)^3
 *    - a rho^2 with eta = b rho / 4.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 discrete velocities (Section II). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

static double g_M[9][9];
static double g_Minv[9][9];
static int g_ready = 0;

/* Moment basis (rho, e, zeta, jx, qx, jy, qy, pxx, pxy) written as the usual
 * polynomials of the discrete velocity, |e|^2 = c2. */
static void build_M(double M[9][9])
{
    for (int a = 0; a < 9; ++a) {
        const double ex = EX[a], ey = EY[a], c2 = ex * ex + ey * ey;
        M[0][a] = 1.0;
        M[1][a] = -4.0 + 3.0 * c2;
        M[2][a] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
        M[3][a] = ex;
        M[4][a] = (-5.0 + 3.0 * c2) * ex;
        M[5][a] = ey;
        M[6][a] = (-5.0 + 3.0 * c2) * ey;
        M[7][a] = ex * ex - ey * ey;
        M[8][a] = ex * ey;
    }
}

/* Gauss-Jordan elimination with partial pivoting: Ainv = A^-1. */
static int invert9(const double A[9][9], double Ainv[9][9])
{
    double W[9][18];
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 18; ++j)
            W[i][j] = (j < 9) ? A[i][j] : (j - 9 == i ? 1.0 : 0.0);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabs(W[r][c]) > fabs(W[piv][c])) piv = r;
        if (W[piv][c] == 0.0) return ORC_EINVAL;
        if (piv != c)
            for (int j = 0; j < 18; ++j) {
                double t = W[c][j];
                W[c][j] = W[piv][j];
                W[piv][j] = t;
            }
        const double d = W[c][c];
        for (int j = 0; j < 18; ++j) W[c][j] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == c) continue;
            const double m = W[r][c];
            if (m == 0.0) continue;
            for (int j = 0; j < 18; ++j) W[r][j] -= m * W[c][j];
        }
    }
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) Ainv[i][j] = W[i][j + 9];
    return ORC_OK;
}

static void ensure_matrices(void)
{
    if (g_ready) return;
#ifdef _OPENMP
#pragma omp critical(orc_matrices)
#endif
    {
        if (!g_ready) {
            build_M(g_M);
            invert9(g_M, g_Minv);
            g_ready = 1;
        }
    }
}

void orc_matrices(double M[81], double Minv[81])
{
    ensure_matrices();
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            M[i * 9 + j] = g_M[i][j];
            Minv[i * 9 + j] = g_Minv[i][j];
        }
}

/* ---------------------------------------------------------------- EOS / psi */

/* Section II: psi = sqrt(2 (p_EOS - rho cs^2) / (G c^2)) with c = 1, cs^2 = 1/3,
 * or the exponential potential psi = psi0 exp(-rho0 / rho) whose EOS is
 * p = rho cs^2 + G c^2 psi^2 / 2.  Eq. (23) is the piecewise-linear EOS. */
int orc_eos(const orc_params *P, double rho, double *p, double *psi)
{
    double pe = 0.0, ps = 0.0;
    if (!(rho > 0.0) || !isfinite(rho)) return ORC_EDOMAIN;
    switch (P->eos_kind) {
    case ORC_EOS_CS: {
        const double a = P->eos[0], b = P->eos[1], R = P->eos[2], T = P->eos[3];
        const double eta = b * rho / 4.0;
        if (!(eta < 1.0)) return ORC_EDOMAIN;
        const double om = 1.0 - eta;
        pe = rho * R * T * (1.0 + eta + eta * eta - eta * eta * eta) / (om * om * om) - a * rho * rho;
        break;
    }
    case ORC_EOS_PIECEWISE: {
        const double thV = P->eos[0], thM = P->eos[1], thL = P->eos[2];
        const double r1 = P->eos[3], r2 = P->eos[4];
        if (rho <= r1)
            pe = rho * thV;
        else if (rho < r2)
            pe = r1 * thV + (rho - r1) * thM;
        else
            pe = r1 * thV + (r2 - r1) * thM + (rho - r2) * thL;
        break;
    }
    case ORC_EOS_EXP: {
        const double psi0 = P->eos[0], rho0 = P->eos[1];
        ps = psi0 * exp(-rho0 / rho);
        /* Section III.A: p0 = rho cs^2 + (G1 + 2 G2) psi^2 / 2 (G2 = 0: Eq. 7) */
        pe = rho / 3.0 + (P->G + 2.0 * P->G2) * ps * ps / 2.0;
        if (p) *p = pe;
        if (psi) *psi = ps;
        return ORC_OK;
    }
    default:
        return ORC_EINVAL;
    }
    if (p) *p = pe; /* the pressure is defined even where psi is not */
    const double Geos = P->G + 2.0 * P->G2;
    if (Geos == 0.0) return ORC_EDOMAIN;
    const double rad = 2.0 * (pe - rho / 3.0) / Geos;
    if (!(rad >= 0.0) || !isfinite(rad)) return ORC_EDOMAIN;
    ps = sqrt(rad);
    if (psi) *psi = ps;
    return ORC_OK;
}

int orc_eos_array(const orc_params *P, long n, const double *rho, double *p, double *psi)
{
    int rc = ORC_OK;
    for (long i = 0; i < n; ++i) {
        double pe = NAN, ps = NAN;
        int r = orc_eos(P, rho[i], &pe, &ps);
        if (r != ORC_OK) rc = r;
        if (p) p[i] = pe;
        if (psi) psi[i] = ps;
    }
    return rc;
}

/* ---------------------------------------------------------- node arithmetic */

static double weight(int a)
{
    /* Eq. (7): w(1) = 1/3 for the axis neighbours, w(2) = 1/12 for the diagonal ones. */
    const int c2 = EX[a] * EX[a] + EY[a] * EY[a];
    return c2 == 1 ? 1.0 / 3.0 : 1.0 / 12.0;
}

void orc_force_and_q(const orc_params *P, const double psi9[9], double F[2], double Q[3])
{
    const double psi = psi9[0];
    double sx = 0.0, sy = 0.0, qxx = 0.0, qyy = 0.0, qxy = 0.0;
    for (int a = 1; a < 9; ++a) {
        const double w = weight(a);
        /* Eq. (7): sum of w psi(x + e) e */
        sx += w * psi9[a] * EX[a];
        sy += w * psi9[a] * EY[a];
        /* Eq. (19): sum of w [psi(x + e) - psi(x)] e e */
        const double d = psi9[a] - psi;
        qxx += w * d * EX[a] * EX[a];
        qyy += w * d * EY[a] * EY[a];
        qxy += w * d * EX[a] * EY[a];
    }
    F[0] = -P->G * psi * sx;
    F[1] = -P->G * psi * sy;
    const double k = P->kappa * P->G / 2.0 * psi;
    Q[0] = k * qxx;
    Q[1] = k * qyy;
    Q[2] = k * qxy;
}

void orc_force_multirange(const orc_params *P, const double psi9[9], const double psi2[9], double F[2],
                          double Q[3])
{
    orc_force_and_q(P, psi9, F, Q);
    /* Eq. (9), second range: - psi(x) G2 sum_a w_a psi(x + 2 e_a) e_a */
    double sx = 0.0, sy = 0.0;
    for (int a = 1; a < 9; ++a) {
        sx += weight(a) * psi2[a] * EX[a];
        sy += weight(a) * psi2[a] * EY[a];
    }
    F[0] += -P->G2 * psi9[0] * sx;
    F[1] += -P->G2 * psi9[0] * sy;
}

void orc_forcing_moments(const orc_params *P, const double v[2], const double F[2],
                         double psi, double S[9])
{
    const double vx = v[0], vy = v[1], Fx = F[0], Fy = F[1];
    const double tau_e = 1.0 / P->s[1];
    /* Eq. (5), with S1 replaced by the improved form of Eq. (8) (dt = 1). */
    double S1 = 6.0 * (vx * Fx + vy * Fy);
    if (P->sigma != 0.0) S1 += 12.0 * P->sigma * (Fx * Fx + Fy * Fy) / (psi * psi * (tau_e - 0.5));
    S[0] = 0.0;
    S[1] = S1;
    S[2] = -S1;
    S[3] = Fx;
    S[4] = -Fx;
    S[5] = Fy;
    S[6] = -Fy;
    S[7] = 2.0 * (vx * Fx - vy * Fy);
    S[8] = vx * Fy + vy * Fx;
}

/* Eq. (18) with the relaxation rates s: tau_e^-1 = s[1], tau_zeta^-1 = s[2],
 * tau_v^-1 = s[7] = s[8]. */
static void source_moments_with(const double s[9], const double Q[3], double C[9])
{
    const double tr = Q[0] + Q[1];
    C[0] = 0.0;
    C[1] = 1.5 * s[1] * tr;
    C[2] = -1.5 * s[2] * tr;
    C[3] = 0.0;
    C[4] = 0.0;
    C[5] = 0.0;
    C[6] = 0.0;
    C[7] = -s[7] * (Q[0] - Q[1]);
    C[8] = -s[8] * Q[2];
}

void orc_source_moments(const orc_params *P, const double Q[3], double C[9])
{
    source_moments_with(P->s, Q, C);
}

void orc_collide_node(const orc_params *P, const double f[9], const double F[2],
                      const double Q[3], double psi, double fstar[9])
{
    ensure_matrices();
    /* Eq. (6): rho = sum f, rho v = sum e f + F / 2 */
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        rho += f[a];
        jx += EX[a] * f[a];
        jy += EY[a] * f[a];
    }
    const double v[2] = {(jx + 0.5 * F[0]) / rho, (jy + 0.5 * F[1]) / rho};
    /* m = M f */
    double m[9];
    for (int i = 0; i < 9; ++i) {
        m[i] = 0.0;
        for (int a = 0; a < 9; ++a) m[i] += g_M[i][a] * f[a];
    }
    /* Eq. (3) */
    const double v2 = v[0] * v[0] + v[1] * v[1];
    const double meq[9] = {rho,
                           rho * (-2.0 + 3.0 * v2),
                           rho * (1.0 - 3.0 * v2),
                           rho * v[0],
                           -rho * v[0],
                           rho * v[1],
                           -rho * v[1],
                           rho * (v[0] * v[0] - v[1] * v[1]),
                           rho * v[0] * v[1]};
    /* Section V.C: the viscosity is a step function of the density, nu_V
     * below the threshold and nu_L at or above it; it sets the rate of the
     * stress moments (and so of their share of C). */
    double s[9];
    for (int i = 0; i < 9; ++i) s[i] = P->s[i];
    if (P->rho_nu > 0.0 && rho < P->rho_nu) s[7] = s[8] = P->s_nu_low;
    double S[9], C[9], ms[9];
    orc_forcing_moments(P, v, F, psi, S);
    source_moments_with(s, Q, C);
    /* Eq. (17) with dt = 1 */
    for (int i = 0; i < 9; ++i)
        ms[i] = m[i] - s[i] * (m[i] - meq[i]) + (1.0 - s[i] / 2.0) * S[i] + C[i];
    /* f* = M^-1 m* */
    for (int a = 0; a < 9; ++a) {
        fstar[a] = 0.0;
        for (int i = 0; i < 9; ++i) fstar[a] += g_Minv[a][i] * ms[i];
    }
}

/* ------------------------------------------------------------- grid helpers */

static int valid(const orc_params *P)
{
    if (!P || P->nx < 1 || P->ny < 1) return 0;
    /* the source term (Eq. 19) is defined for the nearest-neighbour force only */
    if (P->G2 != 0.0 && P->kappa != 0.0) return 0;
    if (P->bc_x != ORC_BC_PERIODIC && P->bc_x != ORC_BC_WALL) return 0;
    if (P->bc_y != ORC_BC_PERIODIC && P->bc_y != ORC_BC_WALL) return 0;
    return 1;
}

/* Coordinate of the psi neighbour along one axis: periodic wrap, or, across a
 * wall, the adjacent fluid node itself (neutral-wetting reading). */
static int psi_coord(int c, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) return ((c % n) + n) % n;
    if (c < 0) return 0;
    if (c >= n) return n - 1;
    return c;
}

static int outside(const orc_params *P, int x, int y)
{
    return (P->bc_x == ORC_BC_WALL && (x < 0 || x >= P->nx)) ||
           (P->bc_y == ORC_BC_WALL && (y < 0 || y >= P->ny));
}

static void gather_psi9(const orc_params *P, const double *psi, int x, int y, double psi9[9])
{
    for (int a = 0; a < 9; ++a) {
        const int xx = psi_coord(x + EX[a], P->nx, P->bc_x);
        const int yy = psi_coord(y + EY[a], P->ny, P->bc_y);
        psi9[a] = psi[(long)yy * P->nx + xx];
    }
}

/* psi at x + 2 e_a (same wrap / clamp rule as the first ring). */
static void gather_psi_ring2(const orc_params *P, const double *psi, int x, int y, double psi2[9])
{
    for (int a = 0; a < 9; ++a) {
        const int xx = psi_coord(x + 2 * EX[a], P->nx, P->bc_x);
        const int yy = psi_coord(y + 2 * EY[a], P->ny, P->bc_y);
        psi2[a] = psi[(long)yy * P->nx + xx];
    }
}

/* Interaction force (Eq. 7, or Eq. 9 when G2 != 0) and Q (Eq. 19) at (x, y). */
static void node_force(const orc_params *P, const double *psi, int x, int y, double psi9[9], double F[2],
                       double Q[3])
{
    gather_psi9(P, psi, x, y, psi9);
    if (P->G2 != 0.0) {
        double psi2[9];
        gather_psi_ring2(P, psi, x, y, psi2);
        orc_force_multirange(P, psi9, psi2, F, Q);
    } else {
        orc_force_and_q(P, psi9, F, Q);
    }
}

static int density_and_psi(const orc_params *P, const double *f, double *rho, double *psi)
{
    const long N = (long)P->nx * P->ny;
    int rc = ORC_OK;
    for (long n = 0; n < N; ++n) {
        double r = 0.0;
        for (int a = 0; a < 9; ++a) r += f[a * N + n];
        rho[n] = r;
        double ps = NAN;
        if (orc_eos(P, r, NULL, &ps) != ORC_OK) rc = ORC_EDOMAIN;
        psi[n] = ps;
    }
    return rc;
}

/* ------------------------------------------------------------------ public */

int orc_init(const orc_params *P, const double *rho, const double *ux, const double *uy,
             double *f)
{
    if (!valid(P) || !rho || !f) return ORC_EINVAL;
    ensure_matrices();
    const long N = (long)P->nx * P->ny;
    for (long n = 0; n < N; ++n) {
        const double r = rho[n];
        const double vx = ux ? ux[n] : 0.0, vy = uy ? uy[n] : 0.0;
        const double v2 = vx * vx + vy * vy;
        const double meq[9] = {r, r * (-2.0 + 3.0 * v2), r * (1.0 - 3.0 * v2), r * vx, -r * vx,
                               r * vy, -r * vy, r * (vx * vx - vy * vy), r * vx * vy};
        for (int a = 0; a < 9; ++a) {
            double s = 0.0;
            for (int i = 0; i < 9; ++i) s += g_Minv[a][i] * meq[i];
            f[a * N + n] = s;
        }
    }
    return ORC_OK;
}

int orc_step(const orc_params *P, const double *fin, double *fout)
{
    if (!valid(P) || !fin || !fout || fin == fout) return ORC_EINVAL;
    ensure_matrices();
    const int nx = P->nx, ny = P->ny;
    const long N = (long)nx * ny;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *psi = (double *)malloc(sizeof(double) * N);
    if (!rho || !psi) {
        free(rho);
        free(psi);
        return ORC_EINVAL;
    }
    int rc = density_and_psi(P, fin, rho, psi);
    if (rc == ORC_OK) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const long n = (long)y * nx + x;
                double psi9[9], F[2], Q[3], f9[9], fs[9];
                node_force(P, psi, x, y, psi9, F, Q);
                for (int a = 0; a < 9; ++a) f9[a] = fin[a * N + n];
                orc_collide_node(P, f9, F, Q, psi9[0], fs);
                /* Eq. (4): f_a(x + e_a, t + 1) = f*_a(x, t); halfway bounce-back
                 * returns a population that would leave through a wall to its
                 * own node in the opposite direction. */
                for (int a = 0; a < 9; ++a) {
                    const int tx = x + EX[a], ty = y + EY[a];
                    if (outside(P, tx, ty)) {
                        fout[OPP[a] * N + n] = fs[a];
                    } else {
                        const int wx = ((tx % nx) + nx) % nx, wy = ((ty % ny) + ny) % ny;
                        fout[a * N + (long)wy * nx + wx] = fs[a];
                    }
                }
            }
        }
    }
    free(rho);
    free(psi);
    return rc;
}

int orc_run(const orc_params *P, double *f, long nsteps)
{
    if (!valid(P) || !f || nsteps < 0) return ORC_EINVAL;
    const long N = (long)P->nx * P->ny;
    double *g = (double *)malloc(sizeof(double) * 9 * N);
    if (!g) return ORC_EINVAL;
    double *a = f, *b = g;
    int rc = ORC_OK;
    for (long t = 0; t < nsteps && rc == ORC_OK; ++t) {
        rc = orc_step(P, a, b);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != f) memcpy(f, a, sizeof(double) * 9 * N);
    free(g);
    return rc;
}

/* f* at one node, with its psi neighbourhood evaluated from the densities of
 * the nodes around it (the same arithmetic orc_step performs). */
static int node_fstar(const orc_params *P, const double *f, int x, int y, double fs[9])
{
    const long N = (long)P->nx * P->ny;
    double psi9[9], psi2[9], F[2], Q[3], f9[9];
    for (int ring = 1; ring <= (P->G2 != 0.0 ? 2 : 1); ++ring)
        for (int a = 0; a < 9; ++a) {
            const int xx = psi_coord(x + ring * EX[a], P->nx, P->bc_x);
            const int yy = psi_coord(y + ring * EY[a], P->ny, P->bc_y);
            const long m = (long)yy * P->nx + xx;
            double r = 0.0;
            for (int b = 0; b < 9; ++b) r += f[b * N + m];
            if (orc_eos(P, r, NULL, ring == 1 ? &psi9[a] : &psi2[a]) != ORC_OK) return ORC_EDOMAIN;
        }
    if (P->G2 != 0.0)
        orc_force_multirange(P, psi9, psi2, F, Q);
    else
        orc_force_and_q(P, psi9, F, Q);
    const long n = (long)y * P->nx + x;
    for (int a = 0; a < 9; ++a) f9[a] = f[a * N + n];
    orc_collide_node(P, f9, F, Q, psi9[0], fs);
    return ORC_OK;
}

int orc_step_sampled(const orc_params *P, const double *f, long n, const long *idx, double *out)
{
    if (!valid(P) || !f || !idx || !out || n < 0) return ORC_EINVAL;
    ensure_matrices();
    const int nx = P->nx, ny = P->ny;
    const long N = (long)nx * ny;
    int rc = ORC_OK;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) reduction(min : rc)
#endif
    for (long k = 0; k < n; ++k) {
        if (idx[k] < 0 || idx[k] >= N) {
            rc = ORC_EINVAL;
            continue;
        }
        const int x = (int)(idx[k] % nx), y = (int)(idx[k] / nx);
        double fs[9];
        for (int a = 0; a < 9; ++a) {
            const int sx = x - EX[a], sy = y - EY[a];
            int r;
            if (outside(P, sx, sy)) {
                /* the population arriving along a was bounced back at this node */
                r = node_fstar(P, f, x, y, fs);
                out[k * 9 + a] = fs[OPP[a]];
            } else {
                const int wx = ((sx % nx) + nx) % nx, wy = ((sy % ny) + ny) % ny;
                r = node_fstar(P, f, wx, wy, fs);
                out[k * 9 + a] = fs[a];
            }
            if (r != ORC_OK) rc = r;
        }
    }
    return rc;
}

int orc_moments(const orc_params *P, const double *f, double *rho, double *ux, double *uy)
{
    if (!valid(P) || !f || !rho) return ORC_EINVAL;
    const int nx = P->nx, ny = P->ny;
    const long N = (long)nx * ny;
    double *psi = (double *)malloc(sizeof(double) * N);
    if (!psi) return ORC_EINVAL;
    int rc = density_and_psi(P, f, rho, psi);
    if (rc == ORC_OK && (ux || uy)) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long n = (long)y * nx + x;
                double psi9[9], F[2], Q[3], jx = 0.0, jy = 0.0;
                node_force(P, psi, x, y, psi9, F, Q);
                for (int a = 0; a < 9; ++a) {
                    jx += EX[a] * f[a * N + n];
                    jy += EY[a] * f[a * N + n];
                }
                if (ux) ux[n] = (jx + 0.5 * F[0]) / rho[n];
                if (uy) uy[n] = (jy + 0.5 * F[1]) / rho[n];
            }
    }
    free(psi);
    return rc;
}

static double axis_dist(double d, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        while (d > 0.5 * n) d -= n;
        while (d < -0.5 * n) d += n;
    }
    return d;
}

int orc_diagnostics(const orc_params *P, const double *f, double cx, double cy,
                    double r_in, double r_out, double out[8])
{
    if (!valid(P) || !f || !out) return ORC_EINVAL;
    const int nx = P->nx, ny = P->ny;
    const long N = (long)nx * ny;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *ux = (double *)malloc(sizeof(double) * N);
    double *uy = (double *)malloc(sizeof(double) * N);
    if (!rho || !ux || !uy) {
        free(rho);
        free(ux);
        free(uy);
        return ORC_EINVAL;
    }
    int rc = orc_moments(P, f, rho, ux, uy);
    double mass = 0.0, sin_ = 0.0, sout = 0.0, pin = 0.0, pout = 0.0, vmax = 0.0;
    long nin = 0, nout = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long n = (long)y * nx + x;
            const double dx = axis_dist(x - cx, nx, P->bc_x), dy = axis_dist(y - cy, ny, P->bc_y);
            const double r = sqrt(dx * dx + dy * dy);
            double p = NAN;
            orc_eos(P, rho[n], &p, NULL);
            mass += rho[n];
            if (r <= r_in) {
                sin_ += rho[n];
                pin += p;
                ++nin;
            }
            if (r >= r_out) {
                sout += rho[n];
                pout += p;
                ++nout;
            }
            const double sp = sqrt(ux[n] * ux[n] + uy[n] * uy[n]);
            if (sp > vmax || isnan(sp)) vmax = sp;
        }
    const double rin = nin ? sin_ / nin : NAN, rout = nout ? sout / nout : NAN;
    out[0] = mass;
    out[1] = rin;
    out[2] = rout;
    out[3] = nin ? pin / nin : NAN;
    out[4] = nout ? pout / nout : NAN;
    out[5] = out[3] - out[4];
    out[6] = sqrt((mass - rout * (double)N) / (M_PI * (rin - rout)));
    out[7] = vmax;
    free(rho);
    free(ux);
    free(uy);
    return rc;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
