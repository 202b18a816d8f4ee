/*
 * Plain FP64 CPU oracle of the two-component extension (see lbm_mc_oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY.  Written to be read against the paper, not to be
 * fast: a dense 9x9 moment transform with M built from the moment
 * polynomials and inverted by Gauss-Jordan elimination, two-array push
 * streaming, and per node, in the paper's order:
 *   densities (Eq. 6) -> psi_s = rho_s -> F_s (Eq. 7) and Q_s (Eq. 19) from the
 *   other component's psi -> mixture velocity u (Eq. 6 with both forces) ->
 *   per component m = M f, m_eq (Eq. 3 with rho_s, u), S (Eq. 5 with u, F_s),
 *   C (Eq. 18 with Q_s) -> m* (Eq. 17) -> f* = M^-1 m* -> streaming (Eq. 4).
 * The OpenMP pragma only splits the node loop across threads.
 */
#include "lbm_mc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

static double g_M[9][9], g_Minv[9][9];
static int g_ready = 0;

/* interaction weights w(1) = 1/3, w(2) = 1/12 (Section II) */
static double w_int(int a) { return a == 0 ? 0.0 : (a <= 4 ? 1.0 / 3.0 : 1.0 / 12.0); }

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

static int invert9(double A[9][9], double Ainv[9][9])
{
    double W[9][18];
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 18; ++j) W[i][j] = j < 9 ? A[i][j] : (j - 9 == i ? 1.0 : 0.0);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabs(W[r][c]) > fabs(W[piv][c])) piv = r;
        if (W[piv][c] == 0.0) return ORC_EINVAL;
        for (int j = 0; j < 18 && piv != c; ++j) {
            const double t = W[c][j];
            W[c][j] = W[piv][j];
            W[piv][j] = t;
        }
        const double d = W[c][c];
        for (int j = 0; j < 18; ++j) W[c][j] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == c) continue;
            const double k = W[r][c];
            for (int j = 0; j < 18; ++j) W[r][j] -= k * W[c][j];
        }
    }
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) Ainv[i][j] = W[i][j + 9];
    return ORC_OK;
}

static void ensure_ready(void)
{
    if (g_ready) return;
    build_M(g_M);
    invert9(g_M, g_Minv);
    g_ready = 1;
}

void orcmc_matrices(double M[81], double Minv[81])
{
    ensure_ready();
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            M[i * 9 + j] = g_M[i][j];
            Minv[i * 9 + j] = g_Minv[i][j];
        }
}

/* Coordinate of a neighbour: periodic wrap, or clamp across a wall (psi beyond
 * a wall is that of the adjacent fluid node). */
static int nb_coord(int c, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) return ((c % n) + n) % n;
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

void orcmc_force_and_q(const orcmc_params *P, double psi_s, const double psi_o9[9], double F[2], double Q[3])
{
    double sx = 0.0, sy = 0.0, qxx = 0.0, qyy = 0.0, qxy = 0.0;
    for (int a = 1; a < 9; ++a) {
        const double w = w_int(a);
        sx += w * psi_o9[a] * EX[a];
        sy += w * psi_o9[a] * EY[a];
        const double d = w * (psi_o9[a] - psi_o9[0]);
        qxx += d * EX[a] * EX[a];
        qyy += d * EY[a] * EY[a];
        qxy += d * EX[a] * EY[a];
    }
    F[0] = -P->G * psi_s * sx;
    F[1] = -P->G * psi_s * sy;
    const double k = P->kappa * 0.5 * P->G * psi_s;
    Q[0] = k * qxx;
    Q[1] = k * qyy;
    Q[2] = k * qxy;
}

void orcmc_collide_node(const orcmc_params *P, const double f[9], const double u[2], const double F[2],
                        const double Q[3], double fstar[9])
{
    ensure_ready();
    double rho = 0.0, m[9], meq[9], S[9], C[9], ms[9];
    for (int a = 0; a < 9; ++a) rho += f[a];
    for (int i = 0; i < 9; ++i) {
        m[i] = 0.0;
        for (int a = 0; a < 9; ++a) m[i] += g_M[i][a] * f[a];
    }
    const double vx = u[0], vy = u[1], v2 = vx * vx + vy * vy;
    /* Eq. (3) with the component's density and the mixture velocity */
    const double eq[9] = {1.0, -2.0 + 3.0 * v2, 1.0 - 3.0 * v2, vx, -vx, vy, -vy, vx * vx - vy * vy, vx * vy};
    for (int i = 0; i < 9; ++i) meq[i] = rho * eq[i];
    /* Eq. (5) with the mixture velocity and the component's force */
    S[0] = 0.0;
    S[1] = 6.0 * (vx * F[0] + vy * F[1]);
    S[2] = -S[1];
    S[3] = F[0];
    S[4] = -F[0];
    S[5] = F[1];
    S[6] = -F[1];
    S[7] = 2.0 * (vx * F[0] - vy * F[1]);
    S[8] = vx * F[1] + vy * F[0];
    /* Eq. (18) with the component's Q */
    C[0] = 0.0;
    C[1] = 1.5 * P->s[1] * (Q[0] + Q[1]);
    C[2] = -1.5 * P->s[2] * (Q[0] + Q[1]);
    C[3] = C[4] = C[5] = C[6] = 0.0;
    C[7] = -P->s[7] * (Q[0] - Q[1]);
    C[8] = -P->s[8] * Q[2];
    /* Eq. (17) */
    for (int i = 0; i < 9; ++i) ms[i] = m[i] - P->s[i] * (m[i] - meq[i]) + (1.0 - 0.5 * P->s[i]) * S[i] + C[i];
    for (int a = 0; a < 9; ++a) {
        fstar[a] = 0.0;
        for (int i = 0; i < 9; ++i) fstar[a] += g_Minv[a][i] * ms[i];
    }
}

static int check(const orcmc_params *P)
{
    if (!P || P->nx < 1 || P->ny < 1) return ORC_EINVAL;
    if ((P->bc_x != ORC_BC_PERIODIC && P->bc_x != ORC_BC_WALL) || (P->bc_y != ORC_BC_PERIODIC && P->bc_y != ORC_BC_WALL))
        return ORC_EINVAL;
    return ORC_OK;
}

int orcmc_init(const orcmc_params *P, const double *rhoA, const double *rhoB, const double *ux, const double *uy,
               double *f)
{
    if (check(P) != ORC_OK || !rhoA || !rhoB || !f) return ORC_EINVAL;
    ensure_ready();
    const long N = (long)P->nx * P->ny;
    for (int s = 0; s < 2; ++s) {
        const double *rho = s ? rhoB : rhoA;
        for (long n = 0; n < N; ++n) {
            const double vx = ux ? ux[n] : 0.0, vy = uy ? uy[n] : 0.0, v2 = vx * vx + vy * vy;
            const double eq[9] = {1.0, -2.0 + 3.0 * v2, 1.0 - 3.0 * v2, vx, -vx, vy, -vy, vx * vx - vy * vy, vx * vy};
            for (int a = 0; a < 9; ++a) {
                double v = 0.0;
                for (int i = 0; i < 9; ++i) v += g_Minv[a][i] * rho[n] * eq[i];
                f[((long)s * 9 + a) * N + n] = v;
            }
        }
    }
    return ORC_OK;
}

/* densities of both components at every node */
static void densities(const orcmc_params *P, const double *f, double *rA, double *rB)
{
    const long N = (long)P->nx * P->ny;
    for (long n = 0; n < N; ++n) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < 9; ++q) {
            a += f[(long)q * N + n];
            b += f[(long)(9 + q) * N + n];
        }
        rA[n] = a;
        rB[n] = b;
    }
}

/* forces, source tensors and mixture velocity of node (x, y); psi_s = rho_s */
static void node_state(const orcmc_params *P, const double *f, const double *rA, const double *rB, int x, int y,
                       double F[2][2], double Q[2][3], double u[2])
{
    const long N = (long)P->nx * P->ny, n = (long)y * P->nx + x;
    double pA[9], pB[9];
    for (int a = 0; a < 9; ++a) {
        const long m = (long)nb_coord(y + EY[a], P->ny, P->bc_y) * P->nx + nb_coord(x + EX[a], P->nx, P->bc_x);
        pA[a] = rA[m];
        pB[a] = rB[m];
    }
    orcmc_force_and_q(P, rA[n], pB, F[0], Q[0]);
    orcmc_force_and_q(P, rB[n], pA, F[1], Q[1]);
    double jx = 0.0, jy = 0.0;
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 9; ++a) {
            const double v = f[((long)s * 9 + a) * N + n];
            jx += EX[a] * v;
            jy += EY[a] * v;
        }
    const double rho = rA[n] + rB[n];
    u[0] = (jx + 0.5 * (F[0][0] + F[1][0])) / rho;
    u[1] = (jy + 0.5 * (F[0][1] + F[1][1])) / rho;
}

static void collide_at(const orcmc_params *P, const double *f, const double *rA, const double *rB, int x, int y,
                       double fs[2][9])
{
    const long N = (long)P->nx * P->ny, n = (long)y * P->nx + x;
    double F[2][2], Q[2][3], u[2];
    node_state(P, f, rA, rB, x, y, F, Q, u);
    for (int s = 0; s < 2; ++s) {
        double fv[9];
        for (int a = 0; a < 9; ++a) fv[a] = f[((long)s * 9 + a) * N + n];
        orcmc_collide_node(P, fv, u, F[s], Q[s], fs[s]);
    }
}

int orcmc_step(const orcmc_params *P, const double *fin, double *fout)
{
    if (check(P) != ORC_OK || !fin || !fout) return ORC_EINVAL;
    ensure_ready();
    const int nx = P->nx, ny = P->ny;
    const long N = (long)nx * ny;
    double *rA = malloc(sizeof(double) * N), *rB = malloc(sizeof(double) * N);
    if (!rA || !rB) {
        free(rA);
        free(rB);
        return ORC_EINVAL;
    }
    densities(P, fin, rA, rB);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fs[2][9];
            collide_at(P, fin, rA, rB, x, y, fs);
            /* Eq. (4): push to x + e_a, or back into the opposite slot across a wall */
            for (int s = 0; s < 2; ++s)
                for (int a = 0; a < 9; ++a) {
                    const int tx = x + EX[a], ty = y + EY[a];
                    const int wall = (P->bc_x == ORC_BC_WALL && (tx < 0 || tx >= nx)) ||
                                     (P->bc_y == ORC_BC_WALL && (ty < 0 || ty >= ny));
                    if (wall)
                        fout[((long)s * 9 + OPP[a]) * N + (long)y * nx + x] = fs[s][a];
                    else
                        fout[((long)s * 9 + a) * N + (long)nb_coord(ty, ny, P->bc_y) * nx + nb_coord(tx, nx, P->bc_x)] =
                            fs[s][a];
                }
        }
    free(rA);
    free(rB);
    return ORC_OK;
}

int orcmc_run(const orcmc_params *P, double *f, long nsteps)
{
    if (check(P) != ORC_OK || !f || nsteps < 0) return ORC_EINVAL;
    const long M = 18L * P->nx * P->ny;
    double *g = malloc(sizeof(double) * M);
    if (!g) return ORC_EINVAL;
    for (long k = 0; k < nsteps; ++k) {
        const int rc = orcmc_step(P, f, g);
        if (rc != ORC_OK) {
            free(g);
            return rc;
        }
        memcpy(f, g, sizeof(double) * M);
    }
    free(g);
    return ORC_OK;
}

int orcmc_step_sampled(const orcmc_params *P, const double *f, long n, const long *idx, double *out)
{
    if (check(P) != ORC_OK || !f || !idx || !out || n < 0) return ORC_EINVAL;
    ensure_ready();
    const int nx = P->nx, ny = P->ny;
    const long N = (long)nx * ny;
    double *rA = malloc(sizeof(double) * N), *rB = malloc(sizeof(double) * N);
    if (!rA || !rB) {
        free(rA);
        free(rB);
        return ORC_EINVAL;
    }
    densities(P, f, rA, rB);
    int rc = ORC_OK;
    for (long k = 0; k < n && rc == ORC_OK; ++k) {
        if (idx[k] < 0 || idx[k] >= N) {
            rc = ORC_EINVAL;
            break;
        }
        const int x = (int)(idx[k] % nx), y = (int)(idx[k] / nx);
        /* the populations arriving at (x, y): from x - e_a, or the node's own
         * opposite population reflected at a wall */
        for (int a = 0; a < 9; ++a) {
            const int sx = x - EX[a], sy = y - EY[a];
            const int wall = (P->bc_x == ORC_BC_WALL && (sx < 0 || sx >= nx)) ||
                             (P->bc_y == ORC_BC_WALL && (sy < 0 || sy >= ny));
            double fs[2][9];
            if (wall) {
                collide_at(P, f, rA, rB, x, y, fs);
                for (int s = 0; s < 2; ++s) out[(k * 2 + s) * 9 + a] = fs[s][OPP[a]];
            } else {
                collide_at(P, f, rA, rB, nb_coord(sx, nx, P->bc_x), nb_coord(sy, ny, P->bc_y), fs);
                for (int s = 0; s < 2; ++s) out[(k * 2 + s) * 9 + a] = fs[s][a];
            }
        }
    }
    free(rA);
    free(rB);
    return rc;
}

int orcmc_moments(const orcmc_params *P, const double *f, double *rhoA, double *rhoB, double *ux, double *uy)
{
    if (check(P) != ORC_OK || !f) return ORC_EINVAL;
    const long N = (long)P->nx * P->ny;
    double *rA = malloc(sizeof(double) * N), *rB = malloc(sizeof(double) * N);
    if (!rA || !rB) {
        free(rA);
        free(rB);
        return ORC_EINVAL;
    }
    densities(P, f, rA, rB);
    for (int y = 0; y < P->ny; ++y)
        for (int x = 0; x < P->nx; ++x) {
            const long n = (long)y * P->nx + x;
            double F[2][2], Q[2][3], u[2];
            node_state(P, f, rA, rB, x, y, F, Q, u);
            if (rhoA) rhoA[n] = rA[n];
            if (rhoB) rhoB[n] = rB[n];
            if (ux) ux[n] = u[0];
            if (uy) uy[n] = u[1];
        }
    free(rA);
    free(rB);
    return ORC_OK;
}

int orcmc_diagnostics(const orcmc_params *P, const double *f, double cx, double cy, double r_in, double r_out,
                      double out[11])
{
    if (check(P) != ORC_OK || !f || !out) return ORC_EINVAL;
    const long N = (long)P->nx * P->ny;
    double *rA = malloc(sizeof(double) * N), *rB = malloc(sizeof(double) * N), *ux = malloc(sizeof(double) * N),
           *uy = malloc(sizeof(double) * N);
    if (!rA || !rB || !ux || !uy) {
        free(rA);
        free(rB);
        free(ux);
        free(uy);
        return ORC_EINVAL;
    }
    orcmc_moments(P, f, rA, rB, ux, uy);
    double mA = 0, mB = 0, aIn = 0, aOut = 0, bIn = 0, bOut = 0, pIn = 0, pOut = 0, nIn = 0, nOut = 0, vmax = 0;
    for (int y = 0; y < P->ny; ++y)
        for (int x = 0; x < P->nx; ++x) {
            const long n = (long)y * P->nx + x;
            double dx = x - cx, dy = y - cy;
            if (P->bc_x == ORC_BC_PERIODIC) dx -= P->nx * rint(dx / P->nx);
            if (P->bc_y == ORC_BC_PERIODIC) dy -= P->ny * rint(dy / P->ny);
            const double r = sqrt(dx * dx + dy * dy);
            const double p = (rA[n] + rB[n]) / 3.0 + P->G * rA[n] * rB[n];
            mA += rA[n];
            mB += rB[n];
            if (r <= r_in) {
                aIn += rA[n];
                bIn += rB[n];
                pIn += p;
                nIn += 1;
            }
            if (r >= r_out) {
                aOut += rA[n];
                bOut += rB[n];
                pOut += p;
                nOut += 1;
            }
            const double sp = sqrt(ux[n] * ux[n] + uy[n] * uy[n]);
            if (sp > vmax) vmax = sp;
        }
    out[0] = mA;
    out[1] = mB;
    out[2] = nIn > 0 ? aIn / nIn : NAN;
    out[3] = nOut > 0 ? aOut / nOut : NAN;
    out[4] = nIn > 0 ? bIn / nIn : NAN;
    out[5] = nOut > 0 ? bOut / nOut : NAN;
    out[6] = nIn > 0 ? pIn / nIn : NAN;
    out[7] = nOut > 0 ? pOut / nOut : NAN;
    out[8] = out[6] - out[7];
    out[9] = sqrt((mA - out[3] * (double)N) / (M_PI * (out[2] - out[3])));
    out[10] = vmax;
    free(rA);
    free(rB);
    free(ux);
    free(uy);
    return ORC_OK;
}
