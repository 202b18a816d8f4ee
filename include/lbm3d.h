/*
 * lbm3d.h -- C ABI of the three-dimensional (D3Q19) extension of the
 * pseudopotential MRT lattice Boltzmann step with the surface-tension source
 * term (Li & Luo, arXiv:1306.6445; Section VI names 3D as future work).
 *
 * The 3D form (a reading of the paper): for every node x,
 *   rho = sum_a f_a; psi(rho) as in 2D (Section II; Eq. 23)                Eq. (6)
 *   F = -G psi(x) sum_a w_a psi(x+e_a) e_a, w = 1/6 (axes), 1/12 (diagonals) Eq. (7)
 *   Q = kappa G/2 psi(x) sum_a w_a [psi(x+e_a) - psi(x)] e_a e_a            Eq. (19)
 *   v = (sum_a e_a f_a + F/2) / rho                                         Eq. (6)
 *   m* = m - Lambda (m - m_eq) + (I - Lambda/2) S + Lambda M df(dPi)        Eq. (17)
 *   with m_eq = M f_eq (second-order equilibrium), S = M F_Guo, and df the
 *   second-order equilibrium change for the momentum-flux shift
 *   dPi = (3/5) tr(Q) I - Q + 2 sigma |F|^2 / psi^2 I (in 2D the same rule with
 *   3/4 gives Eq. 18 and the Eq. 8 term); sigma = -epsilon / (16 G);
 *   f_a(x + e_a, t + 1) = (M^-1 m*)_a                                       Eq. (4)
 * M is the orthogonal D3Q19 basis of d'Humieres et al. (2002) in the order
 * (rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz,
 * mx, my, mz).
 *
 * Conventions (as lbm.h): velocities e0 = 0; e1..e6 = +x, -x, +y, -y, +z, -z;
 * e7..e18 = (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1),
 * (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).  Host arrays are
 * double, [z][y][x] (x fastest), populations [19][nz][ny][nx], copied.  The
 * caller owns the workspace (>= lbm3d_workspace_bytes, 256-byte aligned;
 * NULL = the library allocates).  Work is enqueued on the stream given at
 * creation; calls returning data synchronise it.  Errors as lbm_status;
 * lbm_last_error() gives the message.  Precisions LBM_FP64 and LBM_FP32 (FP32
 * stores deviations from the rest-state weights at the smallest initial
 * density, as in 2D).  Out of place: each step reads one population buffer
 * and writes the post-collision state into the other, which the next step
 * streams as it reads it (Eq. 4); populations given to or read from the
 * library are always the streamed state f_a(x).
 */
#ifndef LBM3D_MI355X_H
#define LBM3D_MI355X_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_ctx lbm3d_ctx; /* opaque, library-owned */

typedef struct {
    int32_t nx, ny, nz;       /* nodes, each >= 1 */
    int32_t bc_x, bc_y, bc_z; /* LBM_BC_PERIODIC or LBM_BC_BOUNCEBACK (walls at both ends) */
} lbm3d_grid;

/* Rates 1/tau of the moment groups (rho, e, eps, j, q, nu [3pxx, pww, pxy,
 * pyz, pxz], pi [3pixx, piww], m [mx, my, mz]), each in (0, 2); the shear
 * viscosity is (1/s_nu - 1/2)/3. */
typedef struct {
    double s_rho, s_e, s_eps, s_j, s_q, s_nu, s_pi, s_m;
} lbm3d_rates;

/* Host-only check (no device call): LBM_EINVAL for grid sizes < 1, above
 * 2^31 nodes, or whose x-y planes, covered by tiles of 256 nodes (rows of the
 * smallest power of two >= nx within [16, 256]), need more than 2^32 - 1
 * threads per launch (only very thin grids: ny far below the tile's rows),
 * unknown boundaries or EOS, rates outside (0, 2), kappa outside
 * [0, 1), epsilon < 0 or non-finite, G >= 0 with a sqrt pseudopotential,
 * non-physical EOS parameters (as lbm_validate). */
lbm_status lbm3d_validate(const lbm3d_grid *grid, const lbm_eos *eos, double G, const lbm3d_rates *rates,
                          double kappa, double epsilon);

/* Device bytes a context needs (0 on invalid arguments or precision). */
size_t lbm3d_workspace_bytes(const lbm3d_grid *grid, int32_t precision);

lbm_status lbm3d_create(const lbm3d_grid *grid, const lbm_eos *eos, double G, const lbm3d_rates *rates,
                        double kappa, double epsilon, int32_t precision, void *workspace, size_t workspace_bytes,
                        void *stream, lbm3d_ctx **out);

/* f = f_eq(rho, u) on every node (second-order equilibrium); resets the step
 * counter.  rho host [nz][ny][nx], all > 0; ux, uy, uz may be NULL (zero). */
lbm_status lbm3d_init_density(lbm3d_ctx *ctx, const double *rho, const double *ux, const double *uy,
                              const double *uz);

/* Enqueue n >= 0 time steps on the stream (graph replays of 2k steps while
 * at least 2k remain, see lbm3d_set_graph_steps; single launches for the
 * rest). */
lbm_status lbm3d_step(lbm3d_ctx *ctx, int64_t n);

/* Steps per HIP graph: lbm3d_step replays a captured graph of 2k steps (k
 * >= 1; default 8) while at least 2k steps remain and launches the rest one
 * by one; k = 0 launches every step.  Graphs and single launches give the
 * same bits.  LBM_EINVAL outside [0, 4096].  Synchronises. */
lbm_status lbm3d_set_graph_steps(lbm3d_ctx *ctx, int32_t k);

/* Density and Eq. (6) velocity, host [nz][ny][nx]; ux, uy, uz may be NULL.
 * Synchronises; LBM_EDIVERGED when the run has diverged (arrays still written). */
lbm_status lbm3d_moments(lbm3d_ctx *ctx, double *rho, double *ux, double *uy, double *uz);

/* Populations f_a(x, t) at the current step, host [19][nz][ny][nx] FP64
 * (the streamed state, whatever the buffer layout).  Setting them is a
 * checkpoint restore: bit for bit in FP64; in FP32 they are re-encoded as
 * deviations from the base density of the last lbm3d_init_density (0 before
 * any), so a read-back and restore moves each population by at most one
 * rounding of its stored deviation. */
lbm_status lbm3d_get_populations(lbm3d_ctx *ctx, double *f);
lbm_status lbm3d_set_populations(lbm3d_ctx *ctx, const double *f);

/* Checkpoint / resume (checkpoint/resume of the step): the raw population
 * buffer of the current state with the step count and the FP32 base density,
 * so that a restore continues bit for bit in both precisions.
 * lbm3d_state_bytes() gives the size (0 for a NULL context); host_buf is the
 * caller's.  load: LBM_ESTATE when the checkpoint was taken on another grid
 * or precision, LBM_EINVAL when truncated.  Both synchronise. */
size_t lbm3d_state_bytes(const lbm3d_ctx *ctx);
lbm_status lbm3d_save_state(lbm3d_ctx *ctx, void *host_buf, size_t bytes);
lbm_status lbm3d_load_state(lbm3d_ctx *ctx, const void *host_buf, size_t bytes);

/* FP64 drop diagnostics (see lbm_diag): dims = 3, a sphere about (cx, cy, cz)
 * with r_eq = (3 sum(rho - rho_out) / (4 pi (rho_in - rho_out)))^(1/3);
 * dims = 2, a cylinder along z about (cx, cy) with
 * r_eq = sqrt(sum(rho - rho_out) / (pi nz (rho_in - rho_out))).  The Laplace law
 * reads dp = 2 sigma / R for the sphere and sigma / R for the cylinder.
 * Synchronises. */
lbm_status lbm3d_diagnostics(lbm3d_ctx *ctx, int32_t dims, double cx, double cy, double cz, double r_in,
                             double r_out, lbm_diag *out);

/* Advance n >= 1 steps with per-launch HIP events; mean milliseconds of the
 * psi pass and of the collide kernel (fused schedule: psi_ms = 0 and
 * collide_ms the fused kernel).  Synchronises. */
lbm_status lbm3d_time_kernels(lbm3d_ctx *ctx, int64_t n, double *psi_ms, double *collide_ms);

int64_t lbm3d_steps_taken(const lbm3d_ctx *ctx);

/* Step schedule (both give the same bits).  fused = 1 (the default, with a
 * 64 x 8 tile and z_chunk = 64 in FP32, 128 in FP64): one launch per step; a workgroup of
 * tile_x x tile_y threads owns an x-y tile of as many nodes (32 x 8, 32 x 16,
 * 64 x 4, 64 x 8 or 64 x 16) and marches along z through z_chunk planes,
 * computing psi of each plane ahead (tile and a one-node ring) in LDS.
 * fused = 0: a psi pass over all nodes, then the collide pass (the
 * other arguments ignored).  LBM_EINVAL for other values, or a z_chunk so
 * small that a launch would exceed 2^32 threads. */
lbm_status lbm3d_set_schedule(lbm3d_ctx *ctx, int32_t fused, int32_t tile_x, int32_t tile_y, int32_t z_chunk);

/* Schedule autotuner: times `steps` (>= 1) steps of each of eight candidate
 * schedules (fused 64 x 8 with z chunks of 32, 64 and 128 planes, 64 x 4,
 * 32 x 8, 32 x 16 and 64 x 16 with 64, and the two-pass schedule) on the
 * context's own state, which advances by (steps + 1) per candidate, and sets
 * the fastest; the choice goes to the non-NULL outputs.  Every schedule gives
 * the same bits.  Synchronises. */
lbm_status lbm3d_autotune(lbm3d_ctx *ctx, int32_t steps, int32_t *fused, int32_t *tile_x, int32_t *tile_y,
                          int32_t *z_chunk);
void lbm3d_destroy(lbm3d_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
