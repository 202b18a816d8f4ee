/*
 * Plain FP64 CPU oracle of the three-dimensional (D3Q19) extension of the
 * pseudopotential MRT lattice Boltzmann step with the surface-tension source
 * term of Li & Luo (arXiv:1306.6445), which Section VI names as future work.
 *
 * TEST INFRASTRUCTURE ONLY, like lbm_oracle.h: only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * The 3D form is a reading of the paper (the project's design notes derive
 * it): the source term is Lambda M df with df the second-order equilibrium
 * change for the momentum-flux shift dPi = (3/5) tr(Q) I - Q (the same rule
 * gives Eq. 18 in 2D with 3/4), the Eq. (8) term is Lambda M df for the shift
 * 2 sigma |F|^2 / psi^2 I, m_eq = M f_eq and S = M F_Guo (both exact in 2D).
 *
 * Layout of every population array: f[alpha][z][y][x], alpha = 0..18,
 * x fastest; fields [z][y][x].  Velocities: e0 = 0; e1..e6 = +x, -x, +y, -y,
 * +z, -z; e7..e18 = (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1),
 * (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
 * Moment order (d'Humieres et al. 2002): rho, e, eps, jx, qx, jy, qy, jz, qz,
 * 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz.
 */
#ifndef LBM3D_ORACLE_H
#define LBM3D_ORACLE_H

#include "lbm_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny, nz;
    int bc_x, bc_y, bc_z; /* ORC_BC_PERIODIC or ORC_BC_WALL (halfway bounce-back at both ends) */
    int eos_kind;         /* ORC_EOS_* as in 2D */
    double eos[6];
    double G;             /* interaction strength, Eq. (7) with the 3D weights 1/6, 1/12 */
    double s[19];         /* diagonal of Lambda in moment order */
    double kappa;         /* Eq. (19) */
    double sigma;         /* constant of the improved forcing, Eq. (8) */
} orc3_params;

/* M (rows = moments, built from the moment polynomials) and M^-1 (Gauss-Jordan). */
void orc3_matrices(double M[361], double Minv[361]);

/* Second-order BGK equilibrium w_a rho (1 + 3 e.v + 9/2 (e.v)^2 - 3/2 v^2). */
void orc3_feq(double rho, const double v[3], double feq[19]);

/* Velocity-space forcing of Guo et al.: w_a (3 (e - v).F + 9 (e.v)(e.F)). */
void orc3_guo(const double v[3], const double F[3], double g[19]);

/* Second-order equilibrium change for a momentum-flux shift dPi
 * (xx, yy, zz, xy, yz, xz): df_a = w_a dPi : (e_a e_a - I/3) * 9/2. */
void orc3_flux_shift(const double dPi[6], double df[19]);

/* Force (Eq. 7) and source tensor Q (Eq. 19, xx, yy, zz, xy, yz, xz) from
 * psi19[a] = psi(x + e_a). */
void orc3_force_and_q(const orc3_params *P, const double psi19[19], double F[3], double Q[6]);

/* Post-collision populations of one node. */
void orc3_collide_node(const orc3_params *P, const double f[19], const double F[3], const double Q[6],
                       double psi, double fstar[19]);

int orc3_init(const orc3_params *P, const double *rho, const double *ux, const double *uy, const double *uz,
              double *f);
int orc3_step(const orc3_params *P, const double *fin, double *fout);
int orc3_run(const orc3_params *P, double *f, long nsteps);

/* f(t+1) at the listed nodes (idx = (z ny + y) nx + x) from the full f(t);
 * out[k*19 + a]. */
int orc3_step_sampled(const orc3_params *P, const double *f, long n, const long *idx, double *out);

/* Density and Eq. (6) velocity; ux/uy/uz may be NULL. */
int orc3_moments(const orc3_params *P, const double *f, double *rho, double *ux, double *uy, double *uz);

/* Drop diagnostics, out = {mass, rho_in, rho_out, p_in, p_out, dp, r_eq, max_speed}:
 * dims = 3, a sphere about (cx, cy, cz), r_eq = (3 excess / (4 pi drho))^(1/3);
 * dims = 2, a cylinder along z about (cx, cy), r_eq = sqrt(excess / (pi nz drho));
 * excess = sum(rho - rho_out), drho = rho_in - rho_out; minimum-image distances
 * on periodic axes. */
int orc3_diagnostics(const orc3_params *P, const double *f, int dims, double cx, double cy, double cz,
                     double r_in, double r_out, double out[8]);

#ifdef __cplusplus
}
#endif
#endif
