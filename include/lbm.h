/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the D2Q9 pseudopotential
 * (Shan-Chen) multiple-relaxation-time lattice Boltzmann step with the
 * surface-tension source term of Li & Luo, "Achieving tunable surface tension
 * in the pseudopotential lattice Boltzmann modeling of multiphase flows"
 * (arXiv:1306.6445).
 *
 * One time step (Section II and Section IV) is, for every node x:
 *   rho = sum_a f_a                                               Eq. (6)
 *   psi = psi(rho)  (Section II forms; piecewise EOS Eq. (23))
 *   F   = -G psi(x) sum_a w_a psi(x+e_a) e_a                      Eq. (7)
 *   Q   = kappa G/2 psi(x) sum_a w_a [psi(x+e_a) - psi(x)] e_a e_a Eq. (19)
 *   v   = (sum_a e_a f_a + F/2) / rho                            Eq. (6)
 *   m* = m - Lambda (m - m_eq) + (I - Lambda/2) S + C              Eq. (17)
 *        with m_eq Eq. (3), S Eqs. (5) and (8), C Eq. (18)
 *   f_a(x + e_a, t + 1) = (M^-1 m*)_a                              Eq. (4)
 * in lattice units (c = dt = 1, cs^2 = 1/3).
 *
 * Conventions shared by every entry point
 *  - Velocities: e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0), e4=(0,-1),
 *    e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1).
 *  - Host arrays are row-major [y][x] (nx fastest); population arrays are
 *    [9][ny][nx].  Host arrays are always double and are copied; the library
 *    keeps no pointer to them after the call returns.
 *  - Device memory: the caller owns the workspace (any device allocation of
 *    at least lbm_workspace_bytes() bytes, 256-byte aligned) and must keep it
 *    alive until lbm_destroy().  Passing workspace = NULL makes the library
 *    allocate (and later free) its own.
 *  - Stream: work is enqueued on the hipStream_t given at creation (NULL = the
 *    library creates its own stream).  lbm_step() only enqueues; every call
 *    that returns data to the host synchronises the stream first.
 *  - Errors: every call returns an lbm_status; no exception crosses the ABI.
 *    lbm_last_error() describes the most recent failure on this thread.
 *  - A context is not thread-safe: use one context per thread.
 */
#ifndef LBM_MI355X_H
#define LBM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque, library-owned */

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument; nothing was enqueued */
    LBM_ENOMEM = -2,    /* workspace too small or allocation failed */
    LBM_EDEVICE = -3,   /* a HIP runtime call failed */
    LBM_EDIVERGED = -4, /* a run produced rho <= 0, a non-real psi or NaN */
    LBM_ESTATE = -5     /* call not valid in the context's current state */
} lbm_status;

/* Boundary per axis: periodic, or halfway bounce-back (no-slip) walls at both
 * ends.  At a wall the missing psi neighbour takes the psi of the adjacent
 * fluid node (neutral wetting). */
enum { LBM_BC_PERIODIC = 0, LBM_BC_BOUNCEBACK = 1 };

/* Pseudopotential / equation of state (Section II; Eq. (23)):
 *  LBM_EOS_CS        psi = sqrt(2 (p - rho/3) / G), Carnahan-Starling
 *                    p = rho R T (1+eta+eta^2-eta^3)/(1-eta)^3 - a rho^2,
 *                    eta = b rho / 4;            p[] = {a, b, R, T}
 *  LBM_EOS_PIECEWISE psi = sqrt(2 (p - rho/3) / G), p of Eq. (23);
 *                    p[] = {thetaV, thetaM, thetaL, rho1, rho2}
 *  LBM_EOS_SC_EXP    psi = psi0 exp(-rho0 / rho);  p[] = {psi0, rho0}
 *                    (pressure rho/3 + G psi^2 / 2) */
enum { LBM_EOS_CS = 0, LBM_EOS_PIECEWISE = 1, LBM_EOS_SC_EXP = 2 };

/* Storage / arithmetic precision of the populations:
 *  LBM_FP64            populations and all arithmetic in binary64;
 *  LBM_FP32            arithmetic in binary32, populations stored as binary32
 *                      deviations f_a - w_a rho_ref from the rest-state
 *                      weights at a per-run base density rho_ref: the
 *                      smallest density of the field given to
 *                      lbm_init_density / lbm_run_init_density (the lighter
 *                      phase, whose populations are then stored nearly
 *                      exactly), or the value set by
 *                      lbm_run_set_reference_density, which later
 *                      initialisations keep.  The step's density (Eq. 6) is
 *                      a compensated binary32 sum (TwoSum), so no binary64
 *                      arithmetic runs in the step;
 *  LBM_FP32_BF16STORE  arithmetic in binary32, populations stored as bfloat16
 *                      deviations f_a - w_a rho_w, rho_w the density that the
 *                      node which wrote the population (its upwind node x - e_a
 *                      at the previous step, Eq. 4, or x itself across a wall)
 *                      had when it wrote it; rho_w is kept in binary32, one
 *                      array per step parity.  Stores round stochastically with
 *                      bits from a counter hash of (step, node), so the same
 *                      run gives the same bits.
 * Diagnostics (lbm_diagnostics) always reduce in binary64. */
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP32_BF16STORE = 2 };

typedef struct {
    int32_t nx, ny;     /* nodes; nx, ny >= 1 */
    int32_t bc_x, bc_y; /* LBM_BC_* */
} lbm_grid;

typedef struct {
    int32_t kind; /* LBM_EOS_* */
    int32_t reserved;
    double p[6];
} lbm_eos;

/* Diagonal of Lambda (Eq. 1) as rates 1/tau of the moment groups
 * (rho, e, zeta, j, q, nu); j and q are shared by x and y.  Each in (0, 2). */
typedef struct {
    double s_rho, s_e, s_zeta, s_j, s_q, s_nu;
} lbm_rates;

/* One independent run of a batch. */
typedef struct {
    lbm_grid grid;
    lbm_eos eos;
    double G;       /* interaction strength of Eq. (7); < 0 for the sqrt forms */
    lbm_rates rates;
    double kappa;   /* Eq. (19), in [0, 1) */
    double epsilon; /* exponent of the mechanical-stability integral, Eq. (16);
                     * the Eq. (8) constant is sigma = -epsilon / (16 G).
                     * epsilon != 0 requires s_zeta == s_e (Section II). */
} lbm_run_desc;

/* FP64 droplet diagnostics of one run (Section V.A: delta p = p_in - p_out).
 * rho_in  = mean density within distance r_in of (cx, cy),
 * rho_out = mean density at distance >= r_out (minimum-image on periodic axes),
 * p_in / p_out = mean of the bulk pressure p_EOS(rho) over those regions,
 * dp = p_in - p_out,  r_eq = sqrt(sum(rho - rho_out) / (pi (rho_in - rho_out))),
 * max_speed = max |v| with v the Eq. (6) velocity,
 * status = 0, or 1 when the run has diverged. */
typedef struct {
    double mass, rho_in, rho_out, p_in, p_out, dp, r_eq, max_speed;
    int32_t status;
    int32_t reserved;
} lbm_diag;

/* Region of the droplet diagnostics for one run. */
typedef struct {
    double cx, cy, r_in, r_out;
} lbm_region;

/* ------------------------------------------------------------ validation */

/* Host-only check of one run's parameters (no device call).  LBM_EINVAL when
 * nx or ny < 1, an unknown boundary or EOS kind, any rate outside (0, 2),
 * kappa outside [0, 1), epsilon < 0 or non-finite, epsilon != 0 with
 * s_zeta != s_e, G >= 0 with a sqrt pseudopotential, or non-physical EOS
 * parameters (CS: a, b, R, T <= 0; piecewise: rho1 >= rho2 or rho1 <= 0;
 * exponential: psi0 <= 0 or rho0 <= 0). */
lbm_status lbm_validate_run(const lbm_run_desc *run);

/* Same, in the argument form of lbm_create(). */
lbm_status lbm_validate(const lbm_grid *grid, const lbm_eos *eos, double G,
                        const lbm_rates *rates, double kappa, double epsilon);

/* ----------------------------------------------------------- single run */

/* Device bytes a one-run context needs (0 on invalid arguments). */
size_t lbm_workspace_bytes(const lbm_grid *grid, int32_t precision);

/* Create a one-run context.  Validates as lbm_validate(); the populations are
 * undefined until lbm_init_density() or lbm_set_populations(). */
lbm_status lbm_create(const lbm_grid *grid, const lbm_eos *eos, double G,
                      const lbm_rates *rates, double kappa, double epsilon,
                      int32_t precision, void *workspace, size_t workspace_bytes,
                      void *stream, lbm_ctx **out);

/* f = M^-1 m_eq(rho, u) on every node (Eq. 3); resets the step counter to 0.
 * rho: host [ny][nx], all > 0.  ux, uy: host [ny][nx] or NULL for zero. */
lbm_status lbm_init_density(lbm_ctx *ctx, const double *rho, const double *ux,
                            const double *uy);

/* Enqueue n >= 0 time steps of every run in the context (Eqs. 6, 7, 19, 17, 4). */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Density and Eq. (6) velocity of run 0 into host arrays [ny][nx]; ux, uy may
 * be NULL.  Synchronises.  LBM_EDIVERGED when the run has diverged (the arrays
 * are still written). */
lbm_status lbm_moments(lbm_ctx *ctx, double *rho, double *ux, double *uy);

/* Populations f_a(x, t) of the w x h window of one run whose corner is
 * (x0, y0), host [9][h][w] FP64 (x fastest).  On a periodic axis the window
 * wraps (any x0, w <= nx); on a wall axis it must lie inside the grid.
 * LBM_EINVAL otherwise.  Synchronises.  (Reads back a neighbourhood of a
 * large run without copying the whole run.) */
lbm_status lbm_run_get_window(lbm_ctx *ctx, int32_t run, int32_t x0, int32_t y0, int32_t w, int32_t h, double *f);

/* Bulk pressure p = p_EOS(rho) of every node of one run (the pressure whose
 * jump the Laplace law of Section V.A measures: the bulk part of Eq. (20),
 * where the gradient terms vanish; for the exponential potential
 * rho/3 + G psi^2 / 2), rho = sum_a f_a summed in FP64; host [ny][nx] FP64, NaN
 * where rho <= 0.  Synchronises; LBM_EDIVERGED when the run has diverged
 * (the array is still written). */
lbm_status lbm_run_pressure(lbm_ctx *ctx, int32_t run, double *p);

/* Diagnostics of run 0 (see lbm_diag).  Synchronises. */
lbm_status lbm_diagnostics(lbm_ctx *ctx, double cx, double cy, double r_in,
                           double r_out, lbm_diag *out);

/* Populations f_a(x, t) of run 0 at the current step, host [9][ny][nx] FP64
 * (whatever the storage precision).  Synchronises. */
lbm_status lbm_get_populations(lbm_ctx *ctx, double *f);

/* Overwrite the populations of run 0 at the current step from host [9][ny][nx]
 * FP64 (rounded to the storage precision). */
lbm_status lbm_set_populations(lbm_ctx *ctx, const double *f);

/* Steps taken since the last initialisation. */
int64_t lbm_steps_taken(const lbm_ctx *ctx);

/* Checkpoint: the raw population storage of every run, the step counter and
 * (bf16 storage) the writer densities and the rounding seed, so that a
 * restart continues bit for bit.  lbm_state_bytes() gives the size; load
 * requires a context created with the same runs and precision; the tile shape
 * and schedule may differ.  Both synchronise. */
size_t lbm_state_bytes(const lbm_ctx *ctx);
lbm_status lbm_save_state(lbm_ctx *ctx, void *host_buf, size_t bytes);
lbm_status lbm_load_state(lbm_ctx *ctx, const void *host_buf, size_t bytes);

/* Release the context (and the workspace if the library allocated it). */
void lbm_destroy(lbm_ctx *ctx);

/* Message of the most recent failure on the calling thread ("" if none). */
const char *lbm_last_error(void);

/* ---------------------------------------------------------------- batch */

/* Independent runs (uneven grids, own parameters) stepped together: every
 * kernel launch covers the tiles of all runs.  Workspace as for one run. */
size_t lbm_batch_workspace_bytes(int32_t nruns, const lbm_run_desc *runs, int32_t precision);

lbm_status lbm_batch_create(int32_t nruns, const lbm_run_desc *runs, int32_t precision,
                            void *workspace, size_t workspace_bytes, void *stream,
                            lbm_ctx **out);

int32_t lbm_num_runs(const lbm_ctx *ctx);

/* As lbm_init_density / lbm_moments / lbm_get_populations / lbm_set_populations
 * for one run of the batch.  lbm_run_init_density writes the run's equilibrium
 * populations at the context's current step and leaves the shared step counter
 * unchanged (lbm_init_density also resets it to 0). */
lbm_status lbm_run_init_density(lbm_ctx *ctx, int32_t run, const double *rho,
                                const double *ux, const double *uy);
lbm_status lbm_run_moments(lbm_ctx *ctx, int32_t run, double *rho, double *ux, double *uy);
lbm_status lbm_run_get_populations(lbm_ctx *ctx, int32_t run, double *f);
lbm_status lbm_run_set_populations(lbm_ctx *ctx, int32_t run, const double *f);

/* Density rho = sum_a f_a (Eq. 6) of column x of one run, host [ny] FP64
 * (e.g. to follow an interface).  Synchronises. */
lbm_status lbm_run_density_column(lbm_ctx *ctx, int32_t run, int32_t x, double *rho);

/* Diagnostics of every run in one pass: regions[nruns] in, out[nruns] out.
 * Synchronises; returns LBM_EDIVERGED when any run has diverged (each run's
 * out[].status says which). */
lbm_status lbm_batch_diagnostics(lbm_ctx *ctx, const lbm_region *regions, lbm_diag *out);

/* Multi-range interaction potential of Eq. (9) (Section III, after
 * Sbragaglia et al.): F = -psi(x) sum_a w_a [G1 psi(x + e_a) + G2 psi(x + 2 e_a)] e_a,
 * replacing the run's G by G1; the EOS then reads p0 = rho/3 + (G1 + 2 G2) psi^2 / 2,
 * so the sqrt psi forms invert with G1 + 2 G2 (Section III.A).  Needs kappa = 0
 * (Eq. 19 is defined for Eq. 7 only), G1 + 2 G2 < 0 for the sqrt forms, and the
 * two-kernel schedule; the collide tile then carries a two-node psi halo.
 * G2 = 0 restores Eq. (7).  Synchronises. */
lbm_status lbm_run_set_multirange(lbm_ctx *ctx, int32_t run, double G1, double G2);

/* Step-function viscosity of Section V.C (droplet splashing): nodes whose
 * density is below rho_threshold relax the stress moments (p_xx, p_xy, and
 * their part of the source term C, Eq. 18) at s_nu_low = 1/tau_V instead of
 * rates.s_nu, i.e. nu(rho) = nu_V below the threshold and nu_L at or above it.
 * rho_threshold = 0 turns it off (the default).  LBM_EINVAL for a negative or
 * non-finite threshold or s_nu_low outside (0, 2).  Takes effect at the next
 * step; synchronises the stream. */
lbm_status lbm_run_set_viscosity_step(lbm_ctx *ctx, int32_t run, double rho_threshold, double s_nu_low);

/* Base density rho_ref of the FP32 deviation storage of one run (LBM_ESTATE
 * for FP64 and for bf16, whose base is per population): the stored
 * populations are decoded with the old base and re-encoded with the new one.
 * The run keeps this base through later lbm_run_init_density calls (without
 * it, each initialisation takes the smallest initial density).
 * Synchronises. */
lbm_status lbm_run_set_reference_density(lbm_ctx *ctx, int32_t run, double rho_ref);

/* Per-run divergence flags (0 ok, 1 diverged) into status[nruns]. Synchronises. */
lbm_status lbm_run_status(lbm_ctx *ctx, int32_t *status);

/* ------------------------------------------------------------- tuning */

/* Step-graph length: lbm_step() replays a captured HIP graph of 2*k steps
 * (k >= 1; 0 disables graphs and launches every kernel directly).  Default 16. */
lbm_status lbm_set_graph_steps(lbm_ctx *ctx, int32_t k);

/* Tile shape of the step kernels: tx in {32, 64, 128, 256}, ty in {1, 2, 4, 8},
 * 64 <= tx*ty <= 512 threads.  Default 64 x 4.  Rebuilds the work list and drops any
 * captured graph; synchronises. */
lbm_status lbm_set_tile(lbm_ctx *ctx, int32_t tx, int32_t ty);

/* Step schedule.  rows = 0: two kernels per step, in place (density/psi
 * pass, then collide and stream, one node per thread of a tx x ty tile).
 * rows = 1, 2 or 4: one kernel per step, out of place, rows nodes per thread
 * (tiles of tx x rows*ty nodes): each tile computes psi on itself and its
 * halo from the populations of the current state and writes the next state
 * to the second population buffer of the workspace, in the same layout, so
 * the populations cross HBM once each way per step instead of being read
 * twice (bf16 storage: the writer densities of the previous step are staged
 * with the halo, and the tile writes its own for the next step).  Every
 * schedule gives the same bits.  Default: 2.  LBM_EINVAL for other values.
 * Drops any captured graph; synchronises. */
lbm_status lbm_set_fused(lbm_ctx *ctx, int32_t rows);

/* Tile autotuner: times `steps` (>= 2) steps of this context under each
 * candidate schedule and tile shape (two-kernel 64x4, 128x2, 32x8, 256x1, 64x2,
 * 32x4; fused, as tx x ty threads / rows: 64x4 / 1, 64x4 / 2, 64x4 / 4,
 * 128x2 / 2, 128x2 / 4, 256x1 / 4, 32x8 / 2, 64x2 / 4, 256x2 / 4, 128x4 / 2),
 * graph replay included, and keeps the fastest.  The
 * candidates compute the same step, so the timed steps are real work: the
 * state advances by about 16 * (steps + 2 * graph steps).  The chosen shape is
 * written to tx, ty, fused (each may be NULL).  Synchronises. */
lbm_status lbm_autotune(lbm_ctx *ctx, int32_t steps, int32_t *tx, int32_t *ty, int32_t *fused);

/* Work-list order of the tile kernels: 1 (default) gives each of the eight
 * XCDs a contiguous range of tiles, so tiles sharing halo rows share an L2;
 * 0 keeps the hardware's round-robin order.  Drops any captured graph. */
lbm_status lbm_set_xcd_order(lbm_ctx *ctx, int32_t on);

/* ---------------------------------------------------------- measurement */

/* Advance n >= 1 steps with every kernel launched on its own (no graph), each
 * launch carrying its own start/stop HIP events on the context's stream, and
 * return the mean duration in milliseconds of the density/psi kernel and of
 * the collide-stream kernel (with the fused schedule: 0 and the fused step
 * kernel).  Synchronises.  The state advances exactly as with lbm_step(ctx, n). */
lbm_status lbm_time_kernels(lbm_ctx *ctx, int64_t n, double *psi_ms, double *collide_ms);

/* Plain device copy of `bytes` bytes (16-byte multiple, 16-byte aligned
 * pointers) repeated `reps` times on `stream` (NULL = a private stream); mean
 * milliseconds per copy into *ms.  Reference point for the achievable HBM
 * bandwidth and for scaling hardware byte counters. */
lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, int32_t reps, void *stream,
                           double *ms);

/* ------------------------------------------------- allocation-free step */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_step
 * without a context or workspace.  Advances one FP64 run n >= 0 steps in
 * place on the caller's device array f (the two-kernel in-place AA schedule,
 * 64 x 4 tiles), same bits as lbm_step on a context of that run.
 *  - Arguments as lbm_create (validated on the host, LBM_EINVAL before any
 *    device call).
 *  - f: device, FP64, [9][ny][nx] dense, holding the populations at step t0
 *    in the library's in-place layout of parity t0 mod 2: at even t0 slot a
 *    of node x is f_a(x) (the plain array); at odd t0 f_a(x) sits in slot
 *    opp(a) of x - e_a (slot a of x itself when x - e_a lies beyond a wall).
 *    On return (after the stream has run the work) f holds step t0 + n in the
 *    layout of parity (t0 + n) mod 2.
 *  - status: device int32 or NULL; set to 0 at the start of the call and to
 *    1 if a node produced rho <= 0, a non-real psi or NaN.
 *  - stream: hipStream_t (NULL = the null stream).  Only enqueues kernel
 *    launches: no allocation, no host-device copy, no synchronisation.
 *  - Scratch: psi, the run record, the tile list and (status NULL) the flag
 *    live in a file-scope device array of 33 MiB, one per GPU, kept until the
 *    process ends.  Limits: nx ny <= 4,194,304 nodes and ceil(nx/64) ceil(ny/4)
 *    <= 65,536 tiles (LBM_EINVAL beyond).  Calls on one GPU share that array:
 *    calls that overlap on one GPU (other streams, other threads) race. */
lbm_status lbm_step_noalloc(const lbm_grid *grid, const lbm_eos *eos, double G,
                            const lbm_rates *rates, double kappa, double epsilon,
                            double *f, int64_t t0, int64_t n, int32_t *status,
                            void *stream);

#ifdef __cplusplus
}
#endif
#endif
