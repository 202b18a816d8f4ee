/*
 * C ABI of the two-component (binary mixture) extension of the
 * pseudopotential MRT lattice Boltzmann step with the surface-tension source
 * term (Li & Luo, arXiv:1306.6445).  Section VI names multicomponent models as
 * future work and gives no multicomponent form of Eqs. 18-19; the form here
 * is this library's reading:
 *   components A and B, each a D2Q9 MRT fluid with the same rates (Eq. 1);
 *   psi_s = rho_s; only the cross interaction, strength G > 0 (repulsion):
 *     F_s = -G psi_s(x) sum_a w_a psi_o(x + e_a) e_a          (Eq. 7, o = the other)
 *     Q_s = kappa (G/2) psi_s(x) sum_a w_a [psi_o(x + e_a) - psi_o(x)] e_a e_a  (Eq. 19)
 *   mixture velocity u = sum_s (sum_a e_a f^s_a + F_s / 2) / (rho_A + rho_B)   (Eq. 6);
 *   per component Eq. (17) with m_eq of Eq. (3) at (rho_s, u), S of Eq. (5)
 *   with (u, F_s) and C of Eq. (18) with Q_s; streaming (Eq. 4) per component,
 *   halfway bounce-back at walls, psi beyond a wall = psi of the adjacent node.
 * The mixture's flux shift is then (kappa G / 6) sum_s (psi_s lap psi_o I -
 * psi_s grad grad psi_o), the two-component Eq. (22): the tension scales as
 * 1 - kappa and flat-interface compositions do not move.
 *
 * Conventions as in lbm.h: host arrays are copied (row-major [y][x]; the
 * populations [2][9][ny][nx], component A first, directions e0..e8 = rest,
 * +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1)); the caller may pass a
 * device workspace (256-byte aligned, at least lbm_mc_workspace_bytes) and a
 * stream, or NULL for either (the library then allocates / creates them and
 * frees them in lbm_mc_destroy); one context per thread; errors are
 * lbm_status codes with the message in lbm_last_error().
 */
#ifndef LBM_MC_H
#define LBM_MC_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_mc_ctx lbm_mc_ctx;

typedef struct {
    double G;        /* cross interaction strength, > 0 */
    double kappa;    /* Eq. (19), in [0, 1) */
    lbm_rates rates; /* (s_rho, s_e, s_zeta, s_j, s_q, s_nu), each in (0, 2); s_j sets the inter-diffusion */
} lbm_mc_params;

/* FP64 diagnostics of a drop of A (Section V.A's Laplace law for the mixture):
 * masses, mean densities of both components within r_in of (cx, cy) and at
 * r_out or beyond (minimum image on periodic axes), mean bulk pressure
 * p = (rhoA + rhoB)/3 + G rhoA rhoB of both regions, dp = p_in - p_out,
 * r_eq = sqrt(sum(rhoA - rhoA_out) / (pi (rhoA_in - rhoA_out))), max |u|;
 * status 0, or 1 when the run has diverged. */
typedef struct {
    double massA, massB, rhoA_in, rhoA_out, rhoB_in, rhoB_out, p_in, p_out, dp, r_eq, max_speed;
    int32_t status, reserved;
} lbm_mc_diag;

/* Host-only check: LBM_EINVAL for nx or ny < 1, more than 2^30 nodes, an
 * unknown boundary, G not finite or <= 0, kappa outside [0, 1), a rate outside
 * (0, 2). */
lbm_status lbm_mc_validate(const lbm_grid *grid, const lbm_mc_params *p);

/* Device bytes a context needs (0 on invalid arguments; precision LBM_FP64 or
 * LBM_FP32 only). */
size_t lbm_mc_workspace_bytes(const lbm_grid *grid, int32_t precision);

/* precision: LBM_FP64, or LBM_FP32 (populations stored as f_a - w_a rho_ref
 * per component, rho_ref the component's smallest initial density; FP32
 * arithmetic with compensated density sums).  LBM_EINVAL for other values. */
lbm_status lbm_mc_create(const lbm_grid *grid, const lbm_mc_params *p, int32_t precision, void *workspace,
                         size_t workspace_bytes, void *stream, lbm_mc_ctx **out);

/* f = M^-1 m_eq(rho_s, u) (Eq. 3) for both components; rhoA, rhoB finite and
 * >= 0 with rhoA + rhoB > 0 at every node; ux, uy may be NULL (zero).  Resets
 * the step count.  Synchronises. */
lbm_status lbm_mc_init_density(lbm_mc_ctx *ctx, const double *rhoA, const double *rhoB, const double *ux,
                               const double *uy);

/* Advance n >= 0 steps (one fused launch each), enqueued on the stream
 * (graph replays of 2k steps while at least 2k remain, see
 * lbm_mc_set_graph_steps; single launches for the rest). */
lbm_status lbm_mc_step(lbm_mc_ctx *ctx, int64_t n);

/* Steps per HIP graph: lbm_mc_step replays a captured graph of 2k steps (k
 * >= 1; default 8) while at least 2k steps remain and launches the rest one
 * by one; k = 0 launches every step.  Graphs and single launches give the
 * same bits.  LBM_EINVAL outside [0, 4096].  Synchronises. */
lbm_status lbm_mc_set_graph_steps(lbm_mc_ctx *ctx, int32_t k);

/* Component densities and the mixture velocity of Eq. (6) (both forces), FP64
 * host [ny][nx]; any output may be NULL.  Synchronises; LBM_EDIVERGED when the
 * run has diverged (arrays still written). */
lbm_status lbm_mc_moments(lbm_mc_ctx *ctx, double *rhoA, double *rhoB, double *ux, double *uy);

/* Populations of the current state (the streamed state f_a(x, t), whatever
 * the buffer layout), host [2][9][ny][nx] FP64 (set: finite).  Setting them
 * is a checkpoint restore: bit for bit in FP64; in FP32 they are re-encoded as
 * deviations from each component's base density of the last
 * lbm_mc_init_density (0 before any), so a read-back and restore moves each
 * population by at most one rounding of its stored deviation. */
lbm_status lbm_mc_get_populations(lbm_mc_ctx *ctx, double *f);
lbm_status lbm_mc_set_populations(lbm_mc_ctx *ctx, const double *f);

/* Checkpoint / resume: the raw population buffer of the current state with
 * the step count and both FP32 base densities, so that a restore continues
 * bit for bit in both precisions.  lbm_mc_state_bytes() gives the size (0 for
 * a NULL context); host_buf is the caller's.  load: LBM_ESTATE when the
 * checkpoint was taken on another grid or precision, LBM_EINVAL when
 * truncated.  Both synchronise. */
size_t lbm_mc_state_bytes(const lbm_mc_ctx *ctx);
lbm_status lbm_mc_save_state(lbm_mc_ctx *ctx, void *host_buf, size_t bytes);
lbm_status lbm_mc_load_state(lbm_mc_ctx *ctx, const void *host_buf, size_t bytes);

/* Diagnostics of a drop of A about (cx, cy) (see lbm_mc_diag).  Synchronises. */
lbm_status lbm_mc_diagnostics(lbm_mc_ctx *ctx, double cx, double cy, double r_in, double r_out, lbm_mc_diag *out);

/* Tile of the fused step: tx x ty threads (tx in {32, 64, 128, 256}, ty in
 * {1, 2, 4, 8}, 64 <= tx ty <= 512), each with `rows` nodes (1, 2 or 4) ty
 * rows apart.  Every shape gives the same bits.  Default one row of 128 x 4
 * threads for FP32, of 64 x 8 for FP64. */
lbm_status lbm_mc_set_tile(lbm_mc_ctx *ctx, int32_t tx, int32_t ty, int32_t rows);

/* Tile autotuner: times `steps` (>= 1) steps of each of ten candidate tiles
 * (128 x 4, 64 x 8, 256 x 2, 64 x 4 with one row; 128 x 4, 64 x 4, 128 x 2,
 * 256 x 2, 64 x 8, 32 x 8 with two) on the context's own state, which
 * advances by (steps + 1) per candidate, and sets the fastest; the choice goes
 * to the non-NULL outputs.  Every tile gives the same bits.  Synchronises. */
lbm_status lbm_mc_autotune(lbm_mc_ctx *ctx, int32_t steps, int32_t *tx, int32_t *ty, int32_t *rows);

/* Advance n >= 1 steps with HIP events around each launch; mean milliseconds
 * per step kernel.  Synchronises. */
lbm_status lbm_mc_time_kernels(lbm_mc_ctx *ctx, int64_t n, double *step_ms);

int64_t lbm_mc_steps_taken(const lbm_mc_ctx *ctx);
void lbm_mc_destroy(lbm_mc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
