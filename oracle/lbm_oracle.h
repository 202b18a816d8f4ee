/*
 * Plain FP64 CPU oracle for the D2Q9 pseudopotential (Shan-Chen) MRT lattice
 * Boltzmann step with the surface-tension source term of Li & Luo,
 * "Achieving tunable surface tension in the pseudopotential lattice Boltzmann
 * modeling of multiphase flows" (arXiv:1306.6445).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and its implementation belong to the
 * oracle: only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with the
 * HIP library, and the HIP library never calls it.
 *
 * Layout of every population array: f[alpha][y][x], alpha = 0..8, row-major,
 * nx*ny nodes per direction.  Every density / velocity field is [y][x].
 * Velocity order (Section II, D2Q9): e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0),
 * e4=(0,-1), e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_EOS_CS = 0, ORC_EOS_PIECEWISE = 1, ORC_EOS_EXP = 2 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1 };

/* Return codes. */
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EDOMAIN = -2 };

typedef struct {
    int nx, ny;
    int bc_x, bc_y;     /* ORC_BC_PERIODIC or ORC_BC_WALL (halfway bounce-back at both ends) */
    int eos_kind;       /* ORC_EOS_* */
    double eos[6];      /* CS: a, b, R, T | PIECEWISE: thetaV, thetaM, thetaL, rho1, rho2 | EXP: psi0, rho0 */
    double G;           /* interaction strength, Eq. (7) */
    double s[9];        /* diagonal of Lambda in moment order (rho,e,zeta,jx,qx,jy,qy,pxx,pxy), Eq. (1) */
    double kappa;       /* Eq. (19) */
    double sigma;       /* constant of the improved forcing, Eq. (8) */
    double rho_nu;      /* step-function viscosity of Section V.C: nodes with rho < rho_nu */
    double s_nu_low;    /* relax p_xx, p_xy at s_nu_low instead of s[7], s[8] (rho_nu = 0: off) */
    double G2;          /* multi-range potential, Eq. (9): G acts as G1 on the neighbours at e_a,
                           G2 on those at 2 e_a; the EOS uses G1 + 2 G2 (Section III.A); needs kappa = 0 */
} orc_params;

/* Transformation matrix M (rows = moments) and its inverse, built at first use. */
void orc_matrices(double M[81], double Minv[81]);

/* p_EOS and psi for one density.  ORC_EDOMAIN when psi is undefined there. */
int orc_eos(const orc_params *P, double rho, double *p, double *psi);
int orc_eos_array(const orc_params *P, long n, const double *rho, double *p, double *psi);

/* Interaction force (Eq. 7) and source tensor (Eq. 19) at one node from the
 * nine psi values of its neighbourhood, psi9[alpha] = psi(x + e_alpha). */
void orc_force_and_q(const orc_params *P, const double psi9[9], double F[2], double Q[3]);

/* Eq. (9): F = -psi(x) sum_a w_a [G psi(x + e_a) + G2 psi(x + 2 e_a)] e_a, with
 * psi2[a] = psi(x + 2 e_a) (psi2[0] unused); Q as in orc_force_and_q. */
void orc_force_multirange(const orc_params *P, const double psi9[9], const double psi2[9], double F[2],
                          double Q[3]);

/* Moment-space forcing S (Eqs. 5 and 8) and source C (Eq. 18). */
void orc_forcing_moments(const orc_params *P, const double v[2], const double F[2],
                         double psi, double S[9]);
void orc_source_moments(const orc_params *P, const double Q[3], double C[9]);

/* Post-collision populations of one node (Eqs. 6, 3, 17, f* = M^-1 m*). */
void orc_collide_node(const orc_params *P, const double f[9], const double F[2],
                      const double Q[3], double psi, double fstar[9]);

/* f = M^-1 m_eq(rho, u) on every node; ux/uy may be NULL (zero velocity). */
int orc_init(const orc_params *P, const double *rho, const double *ux, const double *uy,
             double *f);

/* One full time step: fin at t -> fout at t+1 (two arrays, push streaming, Eq. 4). */
int orc_step(const orc_params *P, const double *fin, double *fout);

/* n steps in place on f (alternating with an internal second array). */
int orc_run(const orc_params *P, double *f, long nsteps);

/* f(t+1) at the listed nodes only, computed from the full state f(t).
 * idx[k] = y*nx + x;  out[k*9 + alpha] = f_alpha(node_k, t+1). */
int orc_step_sampled(const orc_params *P, const double *f, long n, const long *idx, double *out);

/* Density and Eq. (6) velocity on every node; ux/uy may be NULL. */
int orc_moments(const orc_params *P, const double *f, double *rho, double *ux, double *uy);

/* Droplet diagnostics.  out = {mass, rho_in, rho_out, p_in, p_out, dp, r_eq, max_speed}.
 * rho_in = mean density within distance r_in of (cx, cy); rho_out = mean density at
 * distance >= r_out (periodic axes use the minimum-image distance); p = p_EOS;
 * r_eq = sqrt(sum(rho - rho_out) / (pi (rho_in - rho_out))). */
int orc_diagnostics(const orc_params *P, const double *f, double cx, double cy,
                    double r_in, double r_out, double out[8]);

/* Number of OpenMP threads the step loops use (1 when built without OpenMP). */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
