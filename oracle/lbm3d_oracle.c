/*
 * Plain FP64 CPU oracle of the D3Q19 extension (see lbm3d_oracle.h).
 *
 * TEST INFRASTRUCTURE ONLY.  Written to be read against the paper and the
 * derivation of its 3D form, not to be fast: dense 19 x 19 moment products
 * with M built from the moment polynomials and inverted by Gauss-Jordan
 * elimination, the equilibrium, forcing and source moments as M times
 * velocity-space vectors, two-array push streaming.  Per node, in order:
 *   density (Eq. 6) -> psi (Section II; Eq. 23) -> F (Eq. 7) and Q (Eq. 19)
 *   with the 3D weights -> velocity (Eq. 6) -> m = M f, m_eq = M f_eq,
 *   S = M F_Guo (Eq. 5), C = Lambda M df(dPi) with dPi = (3/5) tr Q I - Q
 *   plus the Eq. (8) shift 2 sigma |F|^2 / psi^2 I -> m* (Eq. 17)
 *   -> f* = M^-1 m* -> streaming (Eq. 4) with halfway bounce-back at walls.
 */
#include "lbm3d_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { Q19 = 19 };

static const int E3[Q19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                               {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                               {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static int opp3(int a) { return a == 0 ? 0 : (a % 2 ? a + 1 : a - 1); }

static double c2_of(int a) { return (double)(E3[a][0] * E3[a][0] + E3[a][1] * E3[a][1] + E3[a][2] * E3[a][2]); }

/* equilibrium weights 1/3, 1/18, 1/36 */
static double w_eq(int a)
{
    const double c2 = c2_of(a);
    return c2 == 0.0 ? 1.0 / 3.0 : (c2 == 1.0 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* interaction weights w(1) = 1/6, w(2) = 1/12 (sum w e e = I) */
static double w_int(int a)
{
    const double c2 = c2_of(a);
    return c2 == 0.0 ? 0.0 : (c2 == 1.0 ? 1.0 / 6.0 : 1.0 / 12.0);
}

static double g_M[Q19][Q19], g_Minv[Q19][Q19];
static int g_ready = 0;

/* Rows: rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz,
 * pxz, mx, my, mz as polynomials of the discrete velocity (d'Humieres et al.). */
static void build_M(double M[Q19][Q19])
{
    for (int a = 0; a < Q19; ++a) {
        const double x = E3[a][0], y = E3[a][1], z = E3[a][2], c2 = c2_of(a);
        M[0][a] = 1.0;
        M[1][a] = 19.0 * c2 - 30.0;
        M[2][a] = (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
        M[3][a] = x;
        M[4][a] = (5.0 * c2 - 9.0) * x;
        M[5][a] = y;
        M[6][a] = (5.0 * c2 - 9.0) * y;
        M[7][a] = z;
        M[8][a] = (5.0 * c2 - 9.0) * z;
        M[9][a] = 3.0 * x * x - c2;
        M[10][a] = (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
        M[11][a] = y * y - z * z;
        M[12][a] = (3.0 * c2 - 5.0) * (y * y - z * z);
        M[13][a] = x * y;
        M[14][a] = y * z;
        M[15][a] = x * z;
        M[16][a] = x * (y * y - z * z);
        M[17][a] = y * (z * z - x * x);
        M[18][a] = z * (x * x - y * y);
    }
}

static int invert19(const double A[Q19][Q19], double Ainv[Q19][Q19])
{
    double W[Q19][2 * Q19];
    for (int i = 0; i < Q19; ++i)
        for (int j = 0; j < 2 * Q19; ++j) W[i][j] = j < Q19 ? A[i][j] : (j - Q19 == i ? 1.0 : 0.0);
    for (int c = 0; c < Q19; ++c) {
        int piv = c;
        for (int r = c + 1; r < Q19; ++r)
            if (fabs(W[r][c]) > fabs(W[piv][c])) piv = r;
        if (W[piv][c] == 0.0) return ORC_EINVAL;
        if (piv != c)
            for (int j = 0; j < 2 * Q19; ++j) {
                const double t = W[c][j];
                W[c][j] = W[piv][j];
                W[piv][j] = t;
            }
        const double d = W[c][c];
        for (int j = 0; j < 2 * Q19; ++j) W[c][j] /= d;
        for (int r = 0; r < Q19; ++r) {
            if (r == c) continue;
            const double m = W[r][c];
            if (m == 0.0) continue;
            for (int j = 0; j < 2 * Q19; ++j) W[r][j] -= m * W[c][j];
        }
    }
    for (int i = 0; i < Q19; ++i)
        for (int j = 0; j < Q19; ++j) Ainv[i][j] = W[i][j + Q19];
    return ORC_OK;
}

static void ensure_matrices(void)
{
    if (g_ready) return;
#ifdef _OPENMP
#pragma omp critical(orc3_matrices)
#endif
    {
        if (!g_ready) {
            build_M(g_M);
            invert19(g_M, g_Minv);
            g_ready = 1;
        }
    }
}

void orc3_matrices(double M[361], double Minv[361])
{
    ensure_matrices();
    for (int i = 0; i < Q19; ++i)
        for (int j = 0; j < Q19; ++j) {
            M[i * Q19 + j] = g_M[i][j];
            Minv[i * Q19 + j] = g_Minv[i][j];
        }
}

static void matvec(const double A[Q19][Q19], const double *v, double *out)
{
    for (int i = 0; i < Q19; ++i) {
        double s = 0.0;
        for (int j = 0; j < Q19; ++j) s += A[i][j] * v[j];
        out[i] = s;
    }
}

static double edot(int a, const double v[3]) { return E3[a][0] * v[0] + E3[a][1] * v[1] + E3[a][2] * v[2]; }

void orc3_feq(double rho, const double v[3], double feq[19])
{
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int a = 0; a < Q19; ++a) {
        const double eu = edot(a, v);
        feq[a] = w_eq(a) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * v2);
    }
}

void orc3_guo(const double v[3], const double F[3], double g[19])
{
    for (int a = 0; a < Q19; ++a) {
        const double eu = edot(a, v), eF = edot(a, F);
        const double emv = (E3[a][0] - v[0]) * F[0] + (E3[a][1] - v[1]) * F[1] + (E3[a][2] - v[2]) * F[2];
        g[a] = w_eq(a) * (3.0 * emv + 9.0 * eu * eF);
    }
}

/* dPi : (e e - cs^2 I) / (2 cs^4), cs^2 = 1/3, dPi = (xx, yy, zz, xy, yz, xz) */
void orc3_flux_shift(const double dPi[6], double df[19])
{
    for (int a = 0; a < Q19; ++a) {
        const double x = E3[a][0], y = E3[a][1], z = E3[a][2];
        const double contr = dPi[0] * (x * x - 1.0 / 3.0) + dPi[1] * (y * y - 1.0 / 3.0) +
                             dPi[2] * (z * z - 1.0 / 3.0) + 2.0 * (dPi[3] * x * y + dPi[4] * y * z + dPi[5] * x * z);
        df[a] = w_eq(a) * contr * 4.5;
    }
}

static orc_params eos2d(const orc3_params *P)
{
    orc_params q;
    memset(&q, 0, sizeof(q));
    q.nx = q.ny = 1;
    q.eos_kind = P->eos_kind;
    for (int i = 0; i < 6; ++i) q.eos[i] = P->eos[i];
    q.G = P->G;
    return q;
}

/* Eq. (7) and Eq. (19) with the 3D interaction weights. */
void orc3_force_and_q(const orc3_params *P, const double psi19[19], double F[3], double Q[6])
{
    double s[3] = {0.0, 0.0, 0.0}, q[6] = {0, 0, 0, 0, 0, 0};
    const double p0 = psi19[0];
    for (int a = 1; a < Q19; ++a) {
        const double w = w_int(a), x = E3[a][0], y = E3[a][1], z = E3[a][2];
        s[0] += w * psi19[a] * x;
        s[1] += w * psi19[a] * y;
        s[2] += w * psi19[a] * z;
        const double d = psi19[a] - p0;
        q[0] += w * d * x * x;
        q[1] += w * d * y * y;
        q[2] += w * d * z * z;
        q[3] += w * d * x * y;
        q[4] += w * d * y * z;
        q[5] += w * d * x * z;
    }
    for (int i = 0; i < 3; ++i) F[i] = -P->G * p0 * s[i];
    for (int i = 0; i < 6; ++i) Q[i] = P->kappa * P->G / 2.0 * p0 * q[i];
}

void orc3_collide_node(const orc3_params *P, const double f[19], const double F[3], const double Q[6], double psi,
                       double fstar[19])
{
    ensure_matrices();
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Q19; ++a) {
        rho += f[a];
        for (int i = 0; i < 3; ++i) j[i] += E3[a][i] * f[a];
    }
    /* Eq. (6) velocity */
    double v[3];
    for (int i = 0; i < 3; ++i) v[i] = (j[i] + 0.5 * F[i]) / rho;
    double feq[19], g[19], m[19], meq[19], S[19];
    orc3_feq(rho, v, feq);
    orc3_guo(v, F, g);
    matvec(g_M, f, m);
    matvec(g_M, feq, meq);
    matvec(g_M, g, S);
    /* momentum-flux shifts: the kappa source term and the Eq. (8) term */
    const double trQ = Q[0] + Q[1] + Q[2];
    const double F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    const double iso = 2.0 * P->sigma * F2 / (psi * psi);
    double dPi[6];
    for (int i = 0; i < 3; ++i) dPi[i] = 0.6 * trQ - Q[i] + iso;
    for (int i = 3; i < 6; ++i) dPi[i] = -Q[i];
    double df[19], Cm[19];
    orc3_flux_shift(dPi, df);
    matvec(g_M, df, Cm);
    double ms[19];
    for (int k = 0; k < Q19; ++k)
        ms[k] = m[k] - P->s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * P->s[k]) * S[k] + P->s[k] * Cm[k];
    matvec(g_Minv, ms, fstar);
}

static int nodes3(const orc3_params *P) { return P->nx * P->ny * P->nz; }

static int valid3(const orc3_params *P)
{
    return P && P->nx >= 1 && P->ny >= 1 && P->nz >= 1 &&
           (P->bc_x == ORC_BC_PERIODIC || P->bc_x == ORC_BC_WALL) &&
           (P->bc_y == ORC_BC_PERIODIC || P->bc_y == ORC_BC_WALL) &&
           (P->bc_z == ORC_BC_PERIODIC || P->bc_z == ORC_BC_WALL);
}

int orc3_init(const orc3_params *P, const double *rho, const double *ux, const double *uy, const double *uz,
              double *f)
{
    if (!valid3(P) || !rho || !f) return ORC_EINVAL;
    const long N = nodes3(P);
    for (long n = 0; n < N; ++n) {
        const double v[3] = {ux ? ux[n] : 0.0, uy ? uy[n] : 0.0, uz ? uz[n] : 0.0};
        double feq[19];
        orc3_feq(rho[n], v, feq);
        for (int a = 0; a < Q19; ++a) f[a * N + n] = feq[a];
    }
    return ORC_OK;
}

/* coordinate of a neighbour: periodic wrap, or clamp across a wall */
static int coord(int c, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) return ((c % n) + n) % n;
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

static int density_and_psi(const orc3_params *P, const double *f, double *rho, double *psi)
{
    const long N = nodes3(P);
    const orc_params q = eos2d(P);
    int bad = 0;
    for (long n = 0; n < N; ++n) {
        double s = 0.0;
        for (int a = 0; a < Q19; ++a) s += f[a * N + n];
        rho[n] = s;
        double p;
        if (orc_eos(&q, s, &p, &psi[n]) != ORC_OK) bad = 1;
    }
    return bad ? ORC_EDOMAIN : ORC_OK;
}

static void node_fq(const orc3_params *P, const double *psi, int x, int y, int z, double *p0, double F[3], double Q[6])
{
    double psi19[19];
    for (int a = 0; a < Q19; ++a) {
        const int xx = coord(x + E3[a][0], P->nx, P->bc_x), yy = coord(y + E3[a][1], P->ny, P->bc_y),
                  zz = coord(z + E3[a][2], P->nz, P->bc_z);
        psi19[a] = psi[((long)zz * P->ny + yy) * P->nx + xx];
    }
    *p0 = psi19[0];
    orc3_force_and_q(P, psi19, F, Q);
}

/* post-collision populations of node (x, y, z) streamed into fout (Eq. 4) */
static void collide_and_stream(const orc3_params *P, const double *fin, const double *psi, int x, int y, int z,
                               double *fout)
{
    const long N = nodes3(P);
    const long n = ((long)z * P->ny + y) * P->nx + x;
    double f[19], F[3], Q[6], p0, fs[19];
    for (int a = 0; a < Q19; ++a) f[a] = fin[a * N + n];
    node_fq(P, psi, x, y, z, &p0, F, Q);
    orc3_collide_node(P, f, F, Q, p0, fs);
    for (int a = 0; a < Q19; ++a) {
        const int tx = x + E3[a][0], ty = y + E3[a][1], tz = z + E3[a][2];
        const int wall = (P->bc_x == ORC_BC_WALL && (tx < 0 || tx >= P->nx)) ||
                         (P->bc_y == ORC_BC_WALL && (ty < 0 || ty >= P->ny)) ||
                         (P->bc_z == ORC_BC_WALL && (tz < 0 || tz >= P->nz));
        if (wall) {
            fout[opp3(a) * N + n] = fs[a]; /* halfway bounce-back */
        } else {
            const long t = ((long)coord(tz, P->nz, P->bc_z) * P->ny + coord(ty, P->ny, P->bc_y)) * P->nx +
                           coord(tx, P->nx, P->bc_x);
            fout[a * N + t] = fs[a];
        }
    }
}

int orc3_step(const orc3_params *P, const double *fin, double *fout)
{
    if (!valid3(P) || !fin || !fout) return ORC_EINVAL;
    const long N = nodes3(P);
    double *rho = (double *)malloc(sizeof(double) * N), *psi = (double *)malloc(sizeof(double) * N);
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
        for (int zy = 0; zy < P->nz * P->ny; ++zy)
            for (int x = 0; x < P->nx; ++x) collide_and_stream(P, fin, psi, x, zy % P->ny, zy / P->ny, fout);
    }
    free(rho);
    free(psi);
    return rc;
}

int orc3_run(const orc3_params *P, double *f, long nsteps)
{
    if (!valid3(P) || !f || nsteps < 0) return ORC_EINVAL;
    const long N = nodes3(P);
    double *g = (double *)malloc(sizeof(double) * 19 * N);
    if (!g) return ORC_EINVAL;
    double *a = f, *b = g;
    int rc = ORC_OK;
    for (long s = 0; s < nsteps && rc == ORC_OK; ++s) {
        rc = orc3_step(P, a, b);
        double *t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * 19 * N);
    free(g);
    return rc;
}

int orc3_step_sampled(const orc3_params *P, const double *f, long n, const long *idx, double *out)
{
    if (!valid3(P) || !f || !idx || !out) return ORC_EINVAL;
    const long N = nodes3(P);
    double *rho = (double *)malloc(sizeof(double) * N), *psi = (double *)malloc(sizeof(double) * N);
    if (!rho || !psi) {
        free(rho);
        free(psi);
        return ORC_EINVAL;
    }
    int rc = density_and_psi(P, f, rho, psi);
    for (long k = 0; k < n && rc == ORC_OK; ++k) {
        const long node = idx[k];
        const int x = (int)(node % P->nx), y = (int)((node / P->nx) % P->ny), z = (int)(node / ((long)P->nx * P->ny));
        /* pull: f_a(x, t+1) = f*_a(x - e_a, t), or f*_opp(a)(x, t) across a wall */
        for (int a = 0; a < Q19; ++a) {
            const int sx = x - E3[a][0], sy = y - E3[a][1], sz = z - E3[a][2];
            const int wall = (P->bc_x == ORC_BC_WALL && (sx < 0 || sx >= P->nx)) ||
                             (P->bc_y == ORC_BC_WALL && (sy < 0 || sy >= P->ny)) ||
                             (P->bc_z == ORC_BC_WALL && (sz < 0 || sz >= P->nz));
            int ux = x, uy = y, uz = z, b = opp3(a);
            if (!wall) {
                ux = coord(sx, P->nx, P->bc_x);
                uy = coord(sy, P->ny, P->bc_y);
                uz = coord(sz, P->nz, P->bc_z);
                b = a;
            }
            const long m = ((long)uz * P->ny + uy) * P->nx + ux;
            double fl[19], F[3], Q[6], p0, fs[19];
            for (int c = 0; c < Q19; ++c) fl[c] = f[c * N + m];
            node_fq(P, psi, ux, uy, uz, &p0, F, Q);
            orc3_collide_node(P, fl, F, Q, p0, fs);
            out[k * Q19 + a] = fs[b];
        }
    }
    free(rho);
    free(psi);
    return rc;
}

int orc3_moments(const orc3_params *P, const double *f, double *rho, double *ux, double *uy, double *uz)
{
    if (!valid3(P) || !f || !rho) return ORC_EINVAL;
    const long N = nodes3(P);
    double *psi = (double *)malloc(sizeof(double) * N);
    if (!psi) return ORC_EINVAL;
    int rc = density_and_psi(P, f, rho, psi);
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                const long n = ((long)z * P->ny + y) * P->nx + x;
                double F[3], Q[6], p0, j[3] = {0.0, 0.0, 0.0};
                node_fq(P, psi, x, y, z, &p0, F, Q);
                for (int a = 0; a < Q19; ++a)
                    for (int i = 0; i < 3; ++i) j[i] += E3[a][i] * f[a * N + n];
                if (ux) ux[n] = (j[0] + 0.5 * F[0]) / rho[n];
                if (uy) uy[n] = (j[1] + 0.5 * F[1]) / rho[n];
                if (uz) uz[n] = (j[2] + 0.5 * F[2]) / rho[n];
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

int orc3_diagnostics(const orc3_params *P, const double *f, int dims, double cx, double cy, double cz,
                     double r_in, double r_out, double out[8])
{
    if (!valid3(P) || !f || !out || (dims != 2 && dims != 3)) return ORC_EINVAL;
    const long N = nodes3(P);
    double *rho = (double *)malloc(sizeof(double) * N), *ux = (double *)malloc(sizeof(double) * N),
           *uy = (double *)malloc(sizeof(double) * N), *uz = (double *)malloc(sizeof(double) * N);
    if (!rho || !ux || !uy || !uz) {
        free(rho);
        free(ux);
        free(uy);
        free(uz);
        return ORC_EINVAL;
    }
    int rc = orc3_moments(P, f, rho, ux, uy, uz);
    const orc_params q = eos2d(P);
    double mass = 0.0, sin_ = 0.0, sout = 0.0, pin = 0.0, pout = 0.0, vmax = 0.0;
    long nin = 0, nout = 0;
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                const long n = ((long)z * P->ny + y) * P->nx + x;
                const double dx = axis_dist(x - cx, P->nx, P->bc_x), dy = axis_dist(y - cy, P->ny, P->bc_y);
                const double dz = dims == 3 ? axis_dist(z - cz, P->nz, P->bc_z) : 0.0;
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                double p = NAN, ps;
                orc_eos(&q, rho[n], &p, &ps);
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
                const double sp = sqrt(ux[n] * ux[n] + uy[n] * uy[n] + uz[n] * uz[n]);
                if (sp > vmax || isnan(sp)) vmax = sp;
            }
    const double rin = nin ? sin_ / nin : NAN, rout = nout ? sout / nout : NAN;
    out[0] = mass;
    out[1] = rin;
    out[2] = rout;
    out[3] = nin ? pin / nin : NAN;
    out[4] = nout ? pout / nout : NAN;
    out[5] = out[3] - out[4];
    const double excess = mass - rout * (double)N, drho = rin - rout;
    out[6] = dims == 3 ? cbrt(3.0 * excess / (4.0 * M_PI * drho)) : sqrt(excess / (M_PI * P->nz * drho));
    out[7] = vmax;
    free(rho);
    free(ux);
    free(uy);
    free(uz);
    return rc;
}
