// Host runtime behind the C ABI of include/lbm_mc.h: validation, workspace
// layout, the fused step and the FP64 read-back paths of the two-component
// extension.
#include "../../include/lbm_mc.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_error.hpp"
#include "lbm_trace.hpp"
#include "lbm_mc_kernels.hpp"

namespace {

lbm_status failmc(lbm_status s, const std::string &msg)
{
    lbm::set_last_error(msg);
    return s;
}

#define LBMMC_HIP(call)                                                                                      \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) return failmc(LBM_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// population elements from one direction's array to the next: the nodes
// rounded up to 256 bytes plus a skew of 17 x 256 bytes (as for one component)
int64_t dstride_mc(int64_t nodes, size_t s)
{
    return (int64_t)((((size_t)nodes * s + 255) & ~size_t(255)) + 17 * 256) / (int64_t)s;
}

struct LayoutMC {
    size_t f = 0, f2 = 0, run = 0, status = 0, partial = 0, staging = 0, total = 0;
    int64_t dstride = 0, nblocks = 0;
};

LayoutMC layout_mc(const lbm_grid &g, int prec)
{
    LayoutMC L;
    const int64_t N = (int64_t)g.nx * g.ny;
    const size_t s = prec == LBM_FP64 ? 8 : 4;
    L.dstride = dstride_mc(N, s);
    L.nblocks = (N + lbmmc::kThreadsMC - 1) / lbmmc::kThreadsMC;
    size_t off = 0;
    L.f = off;
    off = al256(off + s * 18 * (size_t)L.dstride);
    L.f2 = off;
    off = al256(off + s * 18 * (size_t)L.dstride);
    L.run = off;
    off = al256(off + sizeof(lbmmc::RunMC));
    L.status = off;
    off = al256(off + sizeof(int32_t));
    L.partial = off;
    off = al256(off + lbmmc::kDiagMC * sizeof(double) * (size_t)L.nblocks);
    L.staging = off;
    off = al256(off + 18 * sizeof(double) * (size_t)N);
    L.total = off;
    return L;
}

lbm_status validate_mc(const lbm_grid *g, const lbm_mc_params *p)
{
    if (!g || !p) return failmc(LBM_EINVAL, "null argument");
    if (g->nx < 1 || g->ny < 1) return failmc(LBM_EINVAL, "nx and ny must be >= 1");
    if ((int64_t)g->nx * g->ny > ((int64_t)1 << 30)) return failmc(LBM_EINVAL, "grid too large for one run");
    for (int bc : {g->bc_x, g->bc_y})
        if (bc != LBM_BC_PERIODIC && bc != LBM_BC_BOUNCEBACK) return failmc(LBM_EINVAL, "unknown boundary kind");
    if (!(std::isfinite(p->G) && p->G > 0.0)) return failmc(LBM_EINVAL, "G must be finite and > 0");
    if (!(p->kappa >= 0.0 && p->kappa < 1.0)) return failmc(LBM_EINVAL, "kappa must lie in [0, 1)");
    const lbm_rates &r = p->rates;
    for (double v : {r.s_rho, r.s_e, r.s_zeta, r.s_j, r.s_q, r.s_nu})
        if (!(v > 0.0 && v < 2.0)) return failmc(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
    // every tile shape must fit one launch
    if (lbmmc::mc_tiles(g->nx, g->ny, 32, 2, 1) > (int64_t)INT32_MAX)
        return failmc(LBM_EINVAL, "grid too large for one run");
    return LBM_OK;
}

int kprec(int p) { return p == LBM_FP64 ? lbmmc::PRECMC_FP64 : lbmmc::PRECMC_FP32; }

} // namespace

struct lbm_mc_ctx {
    int device = 0, precision = LBM_FP64;
    lbm_grid grid{};
    lbmmc::RunMC run{};
    LayoutMC L;
    unsigned char *ws = nullptr;
    bool own_ws = false, own_stream = false;
    hipStream_t stream = nullptr;
    int cur = 0; // population buffer holding the current state
    int64_t steps = 0;
    int tx = 64, ty = 4, rows = 2;
    int graph_k = 8;                  // lbm_mc_step replays HIP graphs of 2 graph_k steps (0: eager)
    int graph_cur = 0;                // buffer the captured graph starts from
    hipGraphExec_t graph = nullptr;
    bool graph_failed = false;
    int64_t nodes() const { return run.nodes; }
    unsigned char *fbuf(int k) { return ws + (k ? L.f2 : L.f); }
    lbmmc::RunMC *drun() { return reinterpret_cast<lbmmc::RunMC *>(ws + L.run); }
    int32_t *dstatus() { return reinterpret_cast<int32_t *>(ws + L.status); }
    double *staging() { return reinterpret_cast<double *>(ws + L.staging); }
    lbmmc::StepMCArgs args()
    {
        lbmmc::StepMCArgs a;
        a.run = drun();
        a.fin = fbuf(cur);
        a.fout = fbuf(cur ^ 1);
        a.status = dstatus();
        a.nx = grid.nx;
        a.ny = grid.ny;
        a.tx = tx;
        a.ty = ty;
        a.rows = rows;
        a.w32 = 18 * (uint64_t)L.dstride * (precision == LBM_FP64 ? 8 : 4) <= 0xffffffffull;
        a.stream = stream;
        return a;
    }
};

namespace {

lbm_status upload_run(lbm_mc_ctx *c)
{
    lbmmc::RunMC &r = c->run;
    r.Gf = (float)r.G;
    r.kappaf = (float)r.kappa;
    for (int k = 0; k < 9; ++k) r.sf[k] = (float)r.s[k];
    for (int s = 0; s < 2; ++s) r.rho_reff[s] = (float)r.rho_ref[s];
    LBMMC_HIP(hipMemcpyAsync(c->drun(), &r, sizeof(lbmmc::RunMC), hipMemcpyHostToDevice, c->stream));
    return LBM_OK;
}

lbm_status read_status(lbm_mc_ctx *c, int32_t &stat)
{
    LBMMC_HIP(hipMemcpyAsync(&stat, c->dstatus(), sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    LBMMC_HIP(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// densities then the mixture velocity of the current state into staging [4][N]
lbm_status moments_to_staging(lbm_mc_ctx *c)
{
    const int64_t N = c->nodes();
    const int p = kprec(c->precision);
    LBMMC_HIP(lbmmc::launch_util_mc(p, 3, c->drun(), c->fbuf(c->cur), nullptr, c->staging(), N, c->stream));
    LBMMC_HIP(lbmmc::launch_util_mc(p, 4, c->drun(), c->fbuf(c->cur), nullptr, c->staging(), N, c->stream));
    return LBM_OK;
}

} // namespace

extern "C" {

lbm_status lbm_mc_validate(const lbm_grid *grid, const lbm_mc_params *p) { return validate_mc(grid, p); }

size_t lbm_mc_workspace_bytes(const lbm_grid *grid, int32_t precision)
{
    if (!grid || grid->nx < 1 || grid->ny < 1) return 0;
    if (precision != LBM_FP64 && precision != LBM_FP32) return 0;
    if ((int64_t)grid->nx * grid->ny > ((int64_t)1 << 30)) return 0;
    return layout_mc(*grid, precision).total;
}

namespace {

void drop_graph_mc(lbm_mc_ctx *c)
{
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

// Captures 2 graph_k steps with the current tile from the current buffer
// (an even number, so the replay ends on the buffer it started from).  A
// failed capture leaves eager stepping in place.
void build_graph_mc(lbm_mc_ctx *c)
{
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        c->graph_failed = true;
        return;
    }
    lbmmc::StepMCArgs a = c->args();
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 * c->graph_k && e == hipSuccess; ++i) {
        e = lbmmc::launch_step_mc(kprec(c->precision), a);
        void *next_in = a.fout; // the buffers alternate
        a.fout = const_cast<void *>(a.fin);
        a.fin = next_in;
    }
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->graph_failed = true;
        return;
    }
    hipError_t e3 = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        c->graph = nullptr;
        (void)hipGetLastError();
        c->graph_failed = true;
        return;
    }
    c->graph_cur = c->cur;
}

} // namespace

void lbm_mc_destroy(lbm_mc_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graph_mc(ctx);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

lbm_status lbm_mc_create(const lbm_grid *grid, const lbm_mc_params *p, int32_t precision, void *workspace,
                         size_t workspace_bytes, void *stream, lbm_mc_ctx **out)
{
    if (!out) return failmc(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    lbm_status s = validate_mc(grid, p);
    if (s != LBM_OK) return s;
    if (precision != LBM_FP64 && precision != LBM_FP32)
        return failmc(LBM_EINVAL, "the two-component model supports LBM_FP64 and LBM_FP32 storage");
    lbm_mc_ctx *c = new (std::nothrow) lbm_mc_ctx;
    if (!c) return failmc(LBM_ENOMEM, "host allocation failed");
    c->precision = precision;
    c->grid = *grid;
    c->L = layout_mc(*grid, precision);
    // fastest shapes of a sweep on a 2048^2 mixture: FP32 128 x 4 threads, one
    // node each; FP64 128 x 2 threads, two nodes each
    // default tiles from a sweep on the 2048^2 mixture: 128 x 4 threads for
    // FP32 and 64 x 8 for FP64, one node each
    c->tx = precision == LBM_FP32 ? 128 : 64;
    c->ty = precision == LBM_FP32 ? 4 : 8;
    c->rows = 1;
    if (workspace && workspace_bytes < c->L.total) {
        delete c;
        return failmc(LBM_ENOMEM, "workspace smaller than lbm_mc_workspace_bytes()");
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
        delete c;
        return failmc(LBM_EINVAL, "workspace must be 256-byte aligned");
    }
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess && stream) {
        c->stream = static_cast<hipStream_t>(stream);
    } else if (e == hipSuccess) {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        c->own_stream = e == hipSuccess;
    }
    if (e == hipSuccess && workspace) {
        c->ws = static_cast<unsigned char *>(workspace);
    } else if (e == hipSuccess) {
        e = hipMalloc(&c->ws, c->L.total);
        c->own_ws = e == hipSuccess;
    }
    if (e != hipSuccess) {
        lbm_mc_destroy(c);
        return failmc(LBM_EDEVICE, std::string("device set-up: ") + hipGetErrorString(e));
    }
    lbmmc::RunMC &r = c->run;
    std::memset(&r, 0, sizeof(r));
    r.nx = grid->nx;
    r.ny = grid->ny;
    r.bc_x = grid->bc_x;
    r.bc_y = grid->bc_y;
    r.nodes = (int64_t)grid->nx * grid->ny;
    r.dstride = c->L.dstride;
    r.G = p->G;
    r.kappa = p->kappa;
    const lbm_rates &q = p->rates;
    const double sv[9] = {q.s_rho, q.s_e, q.s_zeta, q.s_j, q.s_q, q.s_j, q.s_q, q.s_nu, q.s_nu};
    for (int k = 0; k < 9; ++k) r.s[k] = sv[k];
    s = upload_run(c);
    if (s == LBM_OK) {
        hipError_t e2 = hipMemsetAsync(c->dstatus(), 0, sizeof(int32_t), c->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
        if (e2 != hipSuccess) s = failmc(LBM_EDEVICE, std::string("status clear: ") + hipGetErrorString(e2));
    }
    if (s != LBM_OK) {
        lbm_mc_destroy(c);
        return s;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_mc_init_density(lbm_mc_ctx *ctx, const double *rhoA, const double *rhoB, const double *ux,
                               const double *uy)
{
    lbm::TraceRange trace_("lbm_mc_init_density");
    if (!ctx || !rhoA || !rhoB) return failmc(LBM_EINVAL, "null argument");
    const int64_t N = ctx->nodes();
    double rmin[2] = {HUGE_VAL, HUGE_VAL};
    for (int64_t i = 0; i < N; ++i) {
        if (!(std::isfinite(rhoA[i]) && std::isfinite(rhoB[i]) && rhoA[i] >= 0.0 && rhoB[i] >= 0.0 &&
              rhoA[i] + rhoB[i] > 0.0))
            return failmc(LBM_EINVAL, "densities must be finite, >= 0, with a positive sum");
        if ((ux && !std::isfinite(ux[i])) || (uy && !std::isfinite(uy[i])))
            return failmc(LBM_EINVAL, "velocity must be finite");
        rmin[0] = std::fmin(rmin[0], rhoA[i]);
        rmin[1] = std::fmin(rmin[1], rhoB[i]);
    }
    LBMMC_HIP(hipSetDevice(ctx->device));
    ctx->steps = 0;
    // FP32 deviation storage based at each component's smallest initial density
    for (int s = 0; s < 2; ++s) ctx->run.rho_ref[s] = ctx->precision == LBM_FP32 ? rmin[s] : 0.0;
    lbm_status s = upload_run(ctx);
    if (s != LBM_OK) return s;
    double *st = ctx->staging();
    LBMMC_HIP(hipMemcpyAsync(st, rhoA, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    LBMMC_HIP(hipMemcpyAsync(st + N, rhoB, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    const double *u[2] = {ux, uy};
    for (int i = 0; i < 2; ++i) {
        if (u[i])
            LBMMC_HIP(hipMemcpyAsync(st + (i + 2) * N, u[i], sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
        else
            LBMMC_HIP(hipMemsetAsync(st + (i + 2) * N, 0, sizeof(double) * N, ctx->stream));
    }
    LBMMC_HIP(lbmmc::launch_util_mc(kprec(ctx->precision), 2, ctx->drun(), nullptr, ctx->fbuf(ctx->cur), st, N,
                                    ctx->stream));
    LBMMC_HIP(hipMemsetAsync(ctx->dstatus(), 0, sizeof(int32_t), ctx->stream));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_mc_step(lbm_mc_ctx *ctx, int64_t n)
{
    lbm::TraceRange trace_("lbm_mc_step");
    if (!ctx) return failmc(LBM_EINVAL, "null context");
    if (n < 0) return failmc(LBM_EINVAL, "negative step count");
    LBMMC_HIP(hipSetDevice(ctx->device));
    const int64_t block = 2 * (int64_t)ctx->graph_k;
    if (ctx->graph_k > 0 && !ctx->graph_failed && n >= block) {
        if (ctx->graph && ctx->graph_cur != ctx->cur) drop_graph_mc(ctx); // captured from the other buffer
        if (!ctx->graph) build_graph_mc(ctx);
        if (ctx->graph) {
            while (n >= block) {
                LBMMC_HIP(hipGraphLaunch(ctx->graph, ctx->stream));
                ctx->steps += block;
                n -= block;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        LBMMC_HIP(lbmmc::launch_step_mc(kprec(ctx->precision), ctx->args()));
        ctx->cur ^= 1;
        ++ctx->steps;
    }
    return LBM_OK;
}

lbm_status lbm_mc_set_graph_steps(lbm_mc_ctx *ctx, int32_t k)
{
    if (!ctx) return failmc(LBM_EINVAL, "null context");
    if (k < 0 || k > 4096) return failmc(LBM_EINVAL, "graph steps must lie in [0, 4096]");
    LBMMC_HIP(hipSetDevice(ctx->device));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph_mc(ctx);
    ctx->graph_k = k;
    ctx->graph_failed = false;
    return LBM_OK;
}

int64_t lbm_mc_steps_taken(const lbm_mc_ctx *ctx) { return ctx ? ctx->steps : -1; }

lbm_status lbm_mc_set_tile(lbm_mc_ctx *ctx, int32_t tx, int32_t ty, int32_t rows)
{
    if (!ctx) return failmc(LBM_EINVAL, "null context");
    if (!lbmmc::mc_shape_ok(tx, ty, rows))
        return failmc(LBM_EINVAL, "tile: tx in {32,64,128,256}, ty in {1,2,4,8}, 64 <= tx ty <= 512, rows 1, 2 or 4");
    if (lbmmc::mc_tiles(ctx->grid.nx, ctx->grid.ny, tx, ty, rows) > (int64_t)INT32_MAX)
        return failmc(LBM_EINVAL, "tile too small for this grid");
    ctx->tx = tx;
    ctx->ty = ty;
    ctx->rows = rows;
    LBMMC_HIP(hipSetDevice(ctx->device));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph_mc(ctx); // the captured launches carry the tile
    return LBM_OK;
}

// Times `steps` steps of each candidate tile on the context's own state
// (which advances) and keeps the fastest.
lbm_status lbm_mc_autotune(lbm_mc_ctx *ctx, int32_t steps, int32_t *tx, int32_t *ty, int32_t *rows)
{
    lbm::TraceRange trace_("lbm_mc_autotune");
    if (!ctx) return failmc(LBM_EINVAL, "null context");
    if (steps < 1) return failmc(LBM_EINVAL, "autotune needs at least 1 step per candidate");
    LBMMC_HIP(hipSetDevice(ctx->device));
    struct Cand {
        int tx, ty, rows;
    };
    const Cand cands[] = {{128, 4, 1}, {64, 8, 1}, {128, 4, 2}, {256, 2, 1}, {64, 4, 2},
                          {128, 2, 2}, {256, 2, 2}, {64, 8, 2}, {32, 8, 2}, {64, 4, 1}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LBMMC_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return failmc(LBM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(he));
    }
    const Cand keep = {ctx->tx, ctx->ty, ctx->rows};
    Cand pick = keep;
    float best = 0.f;
    lbm_status rc = LBM_OK;
    for (const Cand &c : cands) {
        if (lbm_mc_set_tile(ctx, c.tx, c.ty, c.rows) != LBM_OK) continue;
        if ((rc = lbm_mc_step(ctx, 1)) != LBM_OK) break; // warm-up
        he = hipEventRecord(e0, ctx->stream);
        if (he == hipSuccess && (rc = lbm_mc_step(ctx, steps)) != LBM_OK) break;
        if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            rc = failmc(LBM_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(he));
            break;
        }
        if (best == 0.f || ms < best) {
            best = ms;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) {
        (void)lbm_mc_set_tile(ctx, keep.tx, keep.ty, keep.rows);
        return rc;
    }
    if ((rc = lbm_mc_set_tile(ctx, pick.tx, pick.ty, pick.rows)) != LBM_OK) return rc;
    if (tx) *tx = pick.tx;
    if (ty) *ty = pick.ty;
    if (rows) *rows = pick.rows;
    return LBM_OK;
}

// Checkpoint layout: a 64-byte header {magic, precision, nx, ny, steps,
// population bytes, the two FP32 base densities, 16 reserved bytes}, then the
// raw population buffer of the current state, so that a restore continues
// bit for bit in either precision.
static const uint32_t kMagicMC = 0x434d424cu; // "LBMC"

static uint64_t state_pop_bytes_mc(const lbm_mc_ctx *c)
{
    return 18 * (uint64_t)c->L.dstride * (c->precision == LBM_FP64 ? 8 : 4);
}

size_t lbm_mc_state_bytes(const lbm_mc_ctx *ctx) { return ctx ? 64 + state_pop_bytes_mc(ctx) : 0; }

lbm_status lbm_mc_save_state(lbm_mc_ctx *ctx, void *host_buf, size_t bytes)
{
    lbm::TraceRange trace_("lbm_mc_save_state");
    if (!ctx || !host_buf) return failmc(LBM_EINVAL, "null argument");
    if (bytes < lbm_mc_state_bytes(ctx)) return failmc(LBM_EINVAL, "buffer smaller than lbm_mc_state_bytes()");
    LBMMC_HIP(hipSetDevice(ctx->device));
    unsigned char *p = static_cast<unsigned char *>(host_buf);
    const uint64_t pb = state_pop_bytes_mc(ctx);
    const uint32_t h[4] = {kMagicMC, (uint32_t)ctx->precision, (uint32_t)ctx->grid.nx, (uint32_t)ctx->grid.ny};
    std::memset(p, 0, 64);
    std::memcpy(p, h, 16);
    std::memcpy(p + 16, &ctx->steps, 8);
    std::memcpy(p + 24, &pb, 8);
    std::memcpy(p + 32, ctx->run.rho_ref, 16);
    LBMMC_HIP(hipMemcpyAsync(p + 64, ctx->fbuf(ctx->cur), pb, hipMemcpyDeviceToHost, ctx->stream));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_mc_load_state(lbm_mc_ctx *ctx, const void *host_buf, size_t bytes)
{
    lbm::TraceRange trace_("lbm_mc_load_state");
    if (!ctx || !host_buf) return failmc(LBM_EINVAL, "null argument");
    if (bytes < 64) return failmc(LBM_EINVAL, "checkpoint too short");
    const unsigned char *p = static_cast<const unsigned char *>(host_buf);
    uint32_t h[4];
    int64_t steps;
    uint64_t pb;
    double ref[2];
    std::memcpy(h, p, 16);
    std::memcpy(&steps, p + 16, 8);
    std::memcpy(&pb, p + 24, 8);
    std::memcpy(ref, p + 32, 16);
    if (h[0] != kMagicMC || h[1] != (uint32_t)ctx->precision || h[2] != (uint32_t)ctx->grid.nx ||
        h[3] != (uint32_t)ctx->grid.ny || pb != state_pop_bytes_mc(ctx) || steps < 0 || !std::isfinite(ref[0]) ||
        !std::isfinite(ref[1]))
        return failmc(LBM_ESTATE, "checkpoint does not match this context");
    if (bytes < 64 + pb) return failmc(LBM_EINVAL, "checkpoint truncated");
    LBMMC_HIP(hipSetDevice(ctx->device));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    ctx->steps = steps;
    for (int k = 0; k < 2; ++k) ctx->run.rho_ref[k] = ref[k];
    lbm_status s = upload_run(ctx);
    if (s != LBM_OK) return s;
    LBMMC_HIP(hipMemcpyAsync(ctx->fbuf(ctx->cur), p + 64, pb, hipMemcpyHostToDevice, ctx->stream));
    LBMMC_HIP(hipMemsetAsync(ctx->dstatus(), 0, sizeof(int32_t), ctx->stream));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_mc_get_populations(lbm_mc_ctx *ctx, double *f)
{
    lbm::TraceRange trace_("lbm_mc_get_populations");
    if (!ctx || !f) return failmc(LBM_EINVAL, "null argument");
    LBMMC_HIP(hipSetDevice(ctx->device));
    const int64_t N = ctx->nodes();
    LBMMC_HIP(lbmmc::launch_util_mc(kprec(ctx->precision), 0, ctx->drun(), ctx->fbuf(ctx->cur), nullptr,
                                    ctx->staging(), N, ctx->stream));
    LBMMC_HIP(hipMemcpyAsync(f, ctx->staging(), sizeof(double) * 18 * N, hipMemcpyDeviceToHost, ctx->stream));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_mc_set_populations(lbm_mc_ctx *ctx, const double *f)
{
    lbm::TraceRange trace_("lbm_mc_set_populations");
    if (!ctx || !f) return failmc(LBM_EINVAL, "null argument");
    const int64_t N = ctx->nodes();
    for (int64_t i = 0; i < 18 * N; ++i)
        if (!std::isfinite(f[i])) return failmc(LBM_EINVAL, "populations must be finite");
    LBMMC_HIP(hipSetDevice(ctx->device));
    LBMMC_HIP(hipMemcpyAsync(ctx->staging(), f, sizeof(double) * 18 * N, hipMemcpyHostToDevice, ctx->stream));
    LBMMC_HIP(lbmmc::launch_util_mc(kprec(ctx->precision), 1, ctx->drun(), nullptr, ctx->fbuf(ctx->cur),
                                    ctx->staging(), N, ctx->stream));
    LBMMC_HIP(hipMemsetAsync(ctx->dstatus(), 0, sizeof(int32_t), ctx->stream));
    LBMMC_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_mc_moments(lbm_mc_ctx *ctx, double *rhoA, double *rhoB, double *ux, double *uy)
{
    lbm::TraceRange trace_("lbm_mc_moments");
    if (!ctx) return failmc(LBM_EINVAL, "null context");
    LBMMC_HIP(hipSetDevice(ctx->device));
    const int64_t N = ctx->nodes();
    lbm_status s = moments_to_staging(ctx);
    if (s != LBM_OK) return s;
    double *outs[4] = {rhoA, rhoB, ux, uy};
    for (int i = 0; i < 4; ++i)
        if (outs[i])
            LBMMC_HIP(hipMemcpyAsync(outs[i], ctx->staging() + i * N, sizeof(double) * N, hipMemcpyDeviceToHost,
                                     ctx->stream));
    int32_t stat = 0;
    s = read_status(ctx, stat);
    if (s != LBM_OK) return s;
    return stat ? failmc(LBM_EDIVERGED, "the run has diverged") : LBM_OK;
}

lbm_status lbm_mc_diagnostics(lbm_mc_ctx *ctx, double cx, double cy, double r_in, double r_out, lbm_mc_diag *out)
{
    lbm::TraceRange trace_("lbm_mc_diagnostics");
    if (!ctx || !out) return failmc(LBM_EINVAL, "null argument");
    for (double v : {cx, cy, r_in, r_out})
        if (!std::isfinite(v)) return failmc(LBM_EINVAL, "diagnostic region must be finite");
    LBMMC_HIP(hipSetDevice(ctx->device));
    lbm_status s = moments_to_staging(ctx);
    if (s != LBM_OK) return s;
    double *partial = reinterpret_cast<double *>(ctx->ws + ctx->L.partial);
    LBMMC_HIP(lbmmc::launch_diag_mc(ctx->drun(), ctx->staging(), cx, cy, r_in, r_out, partial, ctx->nodes(),
                                    ctx->stream));
    std::vector<double> h((size_t)lbmmc::kDiagMC * ctx->L.nblocks);
    LBMMC_HIP(hipMemcpyAsync(h.data(), partial, sizeof(double) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
    int32_t stat = 0;
    s = read_status(ctx, stat);
    if (s != LBM_OK) return s;
    // fixed-order FP64 reduction of the block partials
    double v[lbmmc::kDiagMC] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = 0; b < ctx->L.nblocks; ++b) {
        for (int q = 0; q < lbmmc::kDiagMC - 1; ++q) v[q] += h[lbmmc::kDiagMC * b + q];
        v[lbmmc::kDiagMC - 1] = std::fmax(v[lbmmc::kDiagMC - 1], h[lbmmc::kDiagMC * b + lbmmc::kDiagMC - 1]);
    }
    const double N = (double)ctx->nodes();
    out->massA = v[0];
    out->massB = v[1];
    out->rhoA_in = v[4] > 0 ? v[2] / v[4] : NAN;
    out->rhoB_in = v[4] > 0 ? v[3] / v[4] : NAN;
    out->rhoA_out = v[7] > 0 ? v[5] / v[7] : NAN;
    out->rhoB_out = v[7] > 0 ? v[6] / v[7] : NAN;
    out->p_in = v[4] > 0 ? v[8] / v[4] : NAN;
    out->p_out = v[7] > 0 ? v[9] / v[7] : NAN;
    out->dp = out->p_in - out->p_out;
    out->r_eq = std::sqrt((out->massA - out->rhoA_out * N) / (M_PI * (out->rhoA_in - out->rhoA_out)));
    out->max_speed = v[10];
    out->status = stat;
    out->reserved = 0;
    return stat ? failmc(LBM_EDIVERGED, "the run has diverged") : LBM_OK;
}

lbm_status lbm_mc_time_kernels(lbm_mc_ctx *ctx, int64_t n, double *step_ms)
{
    lbm::TraceRange trace_("lbm_mc_time_kernels");
    if (!ctx || n < 1 || !step_ms) return failmc(LBM_EINVAL, "need n >= 1 and an output");
    LBMMC_HIP(hipSetDevice(ctx->device));
    std::vector<hipEvent_t> ev(2 * n, nullptr);
    lbm_status rc = LBM_OK;
    int64_t made = 0;
    for (; made < 2 * n; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) {
            rc = failmc(LBM_EDEVICE, "hipEventCreate failed");
            break;
        }
    double t = 0.0;
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < n && rc == LBM_OK && e == hipSuccess; ++i) {
        lbmmc::StepMCArgs a = ctx->args();
        a.ev0 = ev[2 * i];
        a.ev1 = ev[2 * i + 1];
        e = lbmmc::launch_step_mc(kprec(ctx->precision), a);
        if (e == hipSuccess) {
            ctx->cur ^= 1;
            ++ctx->steps;
        }
    }
    if (rc == LBM_OK && e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    for (int64_t i = 0; i < n && rc == LBM_OK && e == hipSuccess; ++i) {
        float a1 = 0.f;
        e = hipEventElapsedTime(&a1, ev[2 * i], ev[2 * i + 1]);
        t += a1;
    }
    if (rc == LBM_OK && e != hipSuccess) rc = failmc(LBM_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
    for (int64_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (rc == LBM_OK) *step_ms = t / n;
    return rc;
}

} // extern "C"
