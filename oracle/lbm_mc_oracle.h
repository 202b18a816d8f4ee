/*
 * Plain FP64 CPU oracle of the two-component (binary mixture) extension of
 * the D2Q9 pseudopotential MRT lattice Boltzmann step with the surface-tension
 * source term of Li & Luo (arXiv:1306.6445), which Section VI names as future
 * work.
 *
 * TEST INFRASTRUCTURE ONLY, like lbm_oracle.h: only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * The two-component form is a reading of the paper (the project's design
 * notes derive it).  Components A and B, each a D2Q9 MRT fluid with the same
 * M and Lambda; pseudopotentials psi_A = rho_A, psi_B = rho_B (the original
 * Shan-Chen mixture); only the cross interaction, of strength G > 0:
 *   F_s = -G psi_s(x) sum_a w_a psi_o(x + e_a) e_a              (Eq. 7, o = the other component)
 *   Q_s = kappa (G/2) psi_s(x) sum_a w_a [psi_o(x + e_a) - psi_o(x)] e_a e_a   (Eq. 19)
 *   u   = sum_s (sum_a e_a f^s_a + F_s / 2) / (rho_A + rho_B)    (Eq. 6 for the mixture)
 *   m*_s = m_s - Lambda (m_s - m_eq(rho_s, u)) + (I - Lambda/2) S(u, F_s) + C(Q_s)
 *                                                               (Eqs. 17, 3, 5, 18)
 * and streaming (Eq. 4) per component with halfway bounce-back at walls.
 *
 * Layout: populations f[s][alpha][y][x] (s = 0 for A, 1 for B), x fastest;
 * fields [y][x].  Velocities and moments in the order of the 2D oracle:
 * e0..e8 = rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1); moments
 * (rho, e, zeta, jx, qx, jy, qy, pxx, pxy).
 */
#ifndef LBM_MC_ORACLE_H
#define LBM_MC_ORACLE_H

#include "lbm_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny;
    int bc_x, bc_y; /* ORC_BC_PERIODIC or ORC_BC_WALL (halfway bounce-back at both ends) */
    double G;       /* cross interaction strength, > 0 (repulsion) */
    double s[9];    /* diagonal of Lambda in moment order, both components */
    double kappa;   /* Eq. (19) */
} orcmc_params;

/* M (rows = moments, from the moment polynomials) and M^-1 (Gauss-Jordan). */
void orcmc_matrices(double M[81], double Minv[81]);

/* Force (Eq. 7) and source tensor Q (Eq. 19: xx, yy, xy) on component s from
 * its own psi at x and the other component's psi at x + e_a (psi_o9[0] = at x). */
void orcmc_force_and_q(const orcmc_params *P, double psi_s, const double psi_o9[9], double F[2], double Q[3]);

/* Post-collision populations of one component at one node (Eq. 17). */
void orcmc_collide_node(const orcmc_params *P, const double f[9], const double u[2], const double F[2],
                        const double Q[3], double fstar[9]);

/* f = M^-1 m_eq(rho_s, u) per component from host fields (ux, uy may be NULL). */
int orcmc_init(const orcmc_params *P, const double *rhoA, const double *rhoB, const double *ux, const double *uy,
               double *f);
int orcmc_step(const orcmc_params *P, const double *fin, double *fout);
int orcmc_run(const orcmc_params *P, double *f, long nsteps);

/* f(t+1) at the listed nodes (idx = y nx + x) from the full f(t); out[(k*2 + s)*9 + a]. */
int orcmc_step_sampled(const orcmc_params *P, const double *f, long n, const long *idx, double *out);

/* Component densities and the mixture velocity u (Eq. 6 with both forces);
 * any output may be NULL. */
int orcmc_moments(const orcmc_params *P, const double *f, double *rhoA, double *rhoB, double *ux, double *uy);

/* Drop-of-A diagnostics, out = {massA, massB, rhoA_in, rhoA_out, rhoB_in,
 * rhoB_out, p_in, p_out, dp, r_eq, max_speed}: regions within r_in of
 * (cx, cy) and at r_out or beyond (minimum image on periodic axes); bulk
 * pressure p = (rhoA + rhoB)/3 + G rhoA rhoB; r_eq = sqrt(excess_A / (pi
 * (rhoA_in - rhoA_out))), excess_A = sum(rhoA - rhoA_out); max |u|. */
int orcmc_diagnostics(const orcmc_params *P, const double *f, double cx, double cy, double r_in, double r_out,
                      double out[11]);

#ifdef __cplusplus
}
#endif
#endif
