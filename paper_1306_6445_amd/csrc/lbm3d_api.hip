// Host runtime behind the C ABI of include/lbm3d.h: validation, workspace
// layout, the step schedules (fused, or psi pass and collide pass, each
// storing the post-collision state into the second population buffer) and
// the FP64 read-back paths of the D3Q19 extension.
#include "../../include/lbm3d.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm3d_kernels.hpp"
#include "lbm_error.hpp"
#include "lbm_trace.hpp"

namespace {

lbm_status fail3(lbm_status s, const std::string &msg)
{
    lbm::set_last_error(msg);
    return s;
}

#define LBM3_HIP(call)                                                                                      \
    do {                                                                                                    \
        hipError_t e_ = (call);                                                                             \
        if (e_ != hipSuccess) return fail3(LBM_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// population elements from one direction's array to the next: the nodes
// rounded up to 256 bytes plus a skew of 17 x 256 bytes (as in 2D)
int64_t dstride3(int64_t nodes, size_t s) { return (int64_t)((((size_t)nodes * s + 255) & ~size_t(255)) + 17 * 256) / (int64_t)s; }

struct Layout3 {
    size_t f = 0, f2 = 0, psi = 0, run = 0, status = 0, partial = 0, staging = 0, total = 0;
    int64_t dstride = 0, nblocks = 0;
};

Layout3 layout3(const lbm3d_grid &g, int prec)
{
    Layout3 L;
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const size_t s = prec == LBM_FP64 ? 8 : 4;
    L.dstride = dstride3(N, s);
    L.nblocks = (N + lbm3::kThreads3 - 1) / lbm3::kThreads3;
    size_t off = 0;
    L.f = off;
    off = al256(off + s * 19 * (size_t)L.dstride);
    L.f2 = off;
    off = al256(off + s * 19 * (size_t)L.dstride);
    L.psi = off;
    off = al256(off + s * (size_t)N);
    L.run = off;
    off = al256(off + sizeof(lbm3::Run3));
    L.status = off;
    off = al256(off + sizeof(int32_t));
    L.partial = off;
    off = al256(off + 8 * sizeof(double) * (size_t)L.nblocks);
    L.staging = off;
    off = al256(off + 19 * sizeof(double) * (size_t)N);
    L.total = off;
    return L;
}

lbm_status validate3(const lbm3d_grid *g, const lbm_eos *eos, double G, const lbm3d_rates *s, double kappa,
                     double epsilon)
{
    if (!g || !eos || !s) return fail3(LBM_EINVAL, "null argument");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail3(LBM_EINVAL, "nx, ny and nz must be >= 1");
    if ((int64_t)g->nx * g->ny * g->nz > (int64_t)1 << 31) return fail3(LBM_EINVAL, "grid too large for one run");
    // the collide pass covers x-y in tiles of 256 threads, the fused step (default 64 x 8 tiles, 64
    // planes) in fewer threads: a launch holds at most 2^32 - 1 threads
    if (lbm3::collide3_blocks(g->nx, g->ny, g->nz) * lbm3::kThreads3 > (int64_t)UINT32_MAX ||
        lbm3::fused3_blocks(g->nx, g->ny, g->nz, 64, 8, 64) * 512 > (int64_t)UINT32_MAX)
        return fail3(LBM_EINVAL, "grid too large for one run (the collide tiles of the x-y planes exceed 2^32 threads)");
    for (int bc : {g->bc_x, g->bc_y, g->bc_z})
        if (bc != LBM_BC_PERIODIC && bc != LBM_BC_BOUNCEBACK) return fail3(LBM_EINVAL, "unknown boundary kind");
    for (double v : {s->s_rho, s->s_e, s->s_eps, s->s_j, s->s_q, s->s_nu, s->s_pi, s->s_m})
        if (!(v > 0.0 && v < 2.0)) return fail3(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
    if (!(kappa >= 0.0 && kappa < 1.0)) return fail3(LBM_EINVAL, "kappa must lie in [0, 1)");
    if (!std::isfinite(epsilon) || epsilon < 0.0) return fail3(LBM_EINVAL, "epsilon must be finite and >= 0");
    if (!std::isfinite(G)) return fail3(LBM_EINVAL, "G must be finite");
    for (double v : eos->p)
        if (!std::isfinite(v)) return fail3(LBM_EINVAL, "EOS parameters must be finite");
    const double *p = eos->p;
    switch (eos->kind) {
    case LBM_EOS_CS:
        if (!(p[0] > 0 && p[1] > 0 && p[2] > 0 && p[3] > 0))
            return fail3(LBM_EINVAL, "Carnahan-Starling a, b, R, T must be > 0");
        if (!(G < 0.0)) return fail3(LBM_EINVAL, "the sqrt pseudopotential needs G < 0");
        break;
    case LBM_EOS_PIECEWISE:
        if (!(p[3] > 0 && p[3] < p[4])) return fail3(LBM_EINVAL, "piecewise EOS needs 0 < rho1 < rho2");
        if (!(G < 0.0)) return fail3(LBM_EINVAL, "the sqrt pseudopotential needs G < 0");
        break;
    case LBM_EOS_SC_EXP:
        if (!(p[0] > 0 && p[1] > 0)) return fail3(LBM_EINVAL, "psi0 and rho0 must be > 0");
        if (epsilon != 0.0 && G == 0.0) return fail3(LBM_EINVAL, "epsilon != 0 needs G != 0");
        break;
    default:
        return fail3(LBM_EINVAL, "unknown EOS kind");
    }
    return LBM_OK;
}

int kprec(int p) { return p == LBM_FP64 ? lbm3::PREC3_FP64 : lbm3::PREC3_FP32; }

} // namespace

struct lbm3d_ctx {
    int device = 0, precision = LBM_FP64;
    lbm3d_grid grid{};
    lbm3::Run3 run{};
    Layout3 L;
    unsigned char *ws = nullptr;
    bool own_ws = false, own_stream = false, ref_set = false;
    hipStream_t stream = nullptr;
    int cur = 0; // population buffer holding the current state
    int64_t steps = 0;
    int fused = 1, tile_x = 64, tile_y = 8, zchunk = 64; // schedule (lbm3d_set_schedule)
    int graph_k = 8;                  // lbm3d_step replays HIP graphs of 2 graph_k steps (0: eager)
    int graph_cur = 0;                // buffer the captured graph starts from
    hipGraphExec_t graph = nullptr;
    bool graph_failed = false;
    int64_t nodes() const { return run.nodes; }
    unsigned char *fbuf(int k) { return ws + (k ? L.f2 : L.f); }
    lbm3::Run3 *drun() { return reinterpret_cast<lbm3::Run3 *>(ws + L.run); }
    int32_t *dstatus() { return reinterpret_cast<int32_t *>(ws + L.status); }
    double *staging() { return reinterpret_cast<double *>(ws + L.staging); }
    lbm3::Step3Args args()
    {
        lbm3::Step3Args a;
        a.run = drun();
        a.fin = fbuf(cur);
        a.fout = fbuf(cur ^ 1);
        a.psi = ws + L.psi;
        a.status = dstatus();
        a.nodes = nodes();
        a.nx = grid.nx;
        a.ny = grid.ny;
        a.nz = grid.nz;
        a.fused = fused;
        a.tile_x = tile_x;
        a.tile_y = tile_y;
        a.zchunk = zchunk;
        a.w32 = 19 * (uint64_t)L.dstride * (precision == LBM_FP64 ? 8 : 4) <= 0xffffffffull;
        a.stream = stream;
        return a;
    }
};

namespace {

lbm_status upload_run3(lbm3d_ctx *c)
{
    lbm::finish_rundev(c->run.r);
    for (int k = 0; k < 20; ++k) c->run.sf[k] = (float)c->run.s[k];
    c->run.sig2f = (float)c->run.sig2;
    LBM3_HIP(hipMemcpyAsync(c->drun(), &c->run, sizeof(lbm3::Run3), hipMemcpyHostToDevice, c->stream));
    return LBM_OK;
}

lbm_status psi_refresh(lbm3d_ctx *c)
{
    // the psi pass of a step, alone: psi of the current state (read-backs)
    LBM3_HIP(lbm3::launch_psi3(kprec(c->precision), c->drun(), c->fbuf(c->cur), c->ws + c->L.psi, c->dstatus(),
                               c->nodes(), c->stream));
    return LBM_OK;
}

} // namespace

extern "C" {

lbm_status lbm3d_validate(const lbm3d_grid *grid, const lbm_eos *eos, double G, const lbm3d_rates *rates,
                          double kappa, double epsilon)
{
    return validate3(grid, eos, G, rates, kappa, epsilon);
}

size_t lbm3d_workspace_bytes(const lbm3d_grid *grid, int32_t precision)
{
    if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return 0;
    if (precision != LBM_FP64 && precision != LBM_FP32) return 0;
    return layout3(*grid, precision).total;
}

namespace {

void drop_graph3(lbm3d_ctx *c)
{
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

// Captures 2 graph_k steps of the current schedule from the current buffer
// (an even number, so the replay ends on the buffer it started from).  A
// failed capture leaves eager stepping in place.
void build_graph3(lbm3d_ctx *c)
{
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        c->graph_failed = true;
        return;
    }
    lbm3::Step3Args a = c->args();
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 * c->graph_k && e == hipSuccess; ++i) {
        e = lbm3::launch_step3(kprec(c->precision), a);
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

void lbm3d_destroy(lbm3d_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graph3(ctx);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

lbm_status lbm3d_create(const lbm3d_grid *grid, const lbm_eos *eos, double G, const lbm3d_rates *rates,
                        double kappa, double epsilon, int32_t precision, void *workspace, size_t workspace_bytes,
                        void *stream, lbm3d_ctx **out)
{
    if (!out) return fail3(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    lbm_status s = validate3(grid, eos, G, rates, kappa, epsilon);
    if (s != LBM_OK) return s;
    if (precision != LBM_FP64 && precision != LBM_FP32)
        return fail3(LBM_EINVAL, "3D supports LBM_FP64 and LBM_FP32 storage");
    lbm3d_ctx *c = new (std::nothrow) lbm3d_ctx;
    if (!c) return fail3(LBM_ENOMEM, "host allocation failed");
    c->precision = precision;
    // default z chunk from a sweep on a 256^3 drop: 64 planes in FP32, 128 in FP64
    c->zchunk = precision == LBM_FP64 ? 128 : 64;
    c->grid = *grid;
    c->L = layout3(*grid, precision);
    if (workspace && workspace_bytes < c->L.total) {
        delete c;
        return fail3(LBM_ENOMEM, "workspace smaller than lbm3d_workspace_bytes()");
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
        delete c;
        return fail3(LBM_EINVAL, "workspace must be 256-byte aligned");
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
        lbm3d_destroy(c);
        return fail3(LBM_EDEVICE, std::string("device set-up: ") + hipGetErrorString(e));
    }
    // per-run record: EOS and interaction constants in the 2D record
    lbm::RunDev &r = c->run.r;
    std::memset(&c->run, 0, sizeof(c->run));
    r.nx = grid->nx;
    r.ny = grid->ny;
    r.bc_x = grid->bc_x;
    r.bc_y = grid->bc_y;
    r.pitch = grid->nx;
    r.eos_kind = eos->kind;
    for (int i = 0; i < 6; ++i) r.pd.eos[i] = eos->p[i];
    r.pd.G = G;
    r.pd.G_eos = G;
    r.pd.kappa = kappa;
    r.pd.rho_ref = 0.0;
    c->run.nz = grid->nz;
    c->run.bc_z = grid->bc_z;
    c->run.nodes = (int64_t)grid->nx * grid->ny * grid->nz;
    c->run.dstride = c->L.dstride;
    const double *sv[19] = {&rates->s_rho, &rates->s_e, &rates->s_eps, &rates->s_j, &rates->s_q, &rates->s_j,
                            &rates->s_q,   &rates->s_j, &rates->s_q,   &rates->s_nu, &rates->s_pi, &rates->s_nu,
                            &rates->s_pi,  &rates->s_nu, &rates->s_nu, &rates->s_nu, &rates->s_m, &rates->s_m,
                            &rates->s_m};
    for (int k = 0; k < 19; ++k) c->run.s[k] = *sv[k];
    // sigma = -epsilon / (16 G) (Eq. 8 and Eq. 16); the flux shift is 2 sigma |F|^2 / psi^2
    c->run.sig2 = epsilon == 0.0 ? 0.0 : 2.0 * (-epsilon / (16.0 * G));
    s = upload_run3(c);
    if (s == LBM_OK) {
        hipError_t e2 = hipMemsetAsync(c->dstatus(), 0, sizeof(int32_t), c->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
        if (e2 != hipSuccess) s = fail3(LBM_EDEVICE, std::string("status clear: ") + hipGetErrorString(e2));
    }
    if (s != LBM_OK) {
        lbm3d_destroy(c);
        return s;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm3d_init_density(lbm3d_ctx *ctx, const double *rho, const double *ux, const double *uy,
                              const double *uz)
{
    lbm::TraceRange trace_("lbm3d_init_density");
    if (!ctx || !rho) return fail3(LBM_EINVAL, "null argument");
    const int64_t N = ctx->nodes();
    double rmin = HUGE_VAL;
    for (int64_t i = 0; i < N; ++i) {
        if (!(rho[i] > 0.0) || !std::isfinite(rho[i])) return fail3(LBM_EINVAL, "density must be finite and > 0");
        if ((ux && !std::isfinite(ux[i])) || (uy && !std::isfinite(uy[i])) || (uz && !std::isfinite(uz[i])))
            return fail3(LBM_EINVAL, "velocity must be finite");
        rmin = std::fmin(rmin, rho[i]);
    }
    LBM3_HIP(hipSetDevice(ctx->device));
    ctx->steps = 0;
    // FP32 deviation storage based at the lighter phase (the smallest initial density)
    ctx->run.r.pd.rho_ref = ctx->precision == LBM_FP32 ? rmin : 0.0;
    lbm_status s = upload_run3(ctx);
    if (s != LBM_OK) return s;
    double *st = ctx->staging();
    LBM3_HIP(hipMemcpyAsync(st, rho, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    const double *u[3] = {ux, uy, uz};
    for (int i = 0; i < 3; ++i) {
        if (u[i])
            LBM3_HIP(hipMemcpyAsync(st + (i + 1) * N, u[i], sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
        else
            LBM3_HIP(hipMemsetAsync(st + (i + 1) * N, 0, sizeof(double) * N, ctx->stream));
    }
    LBM3_HIP(lbm3::launch_util3(kprec(ctx->precision), 3, ctx->drun(), nullptr, ctx->fbuf(ctx->cur), nullptr, st, N,
                                ctx->stream));
    LBM3_HIP(hipMemsetAsync(ctx->dstatus(), 0, sizeof(int32_t), ctx->stream));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm3d_step(lbm3d_ctx *ctx, int64_t n)
{
    lbm::TraceRange trace_("lbm3d_step");
    if (!ctx) return fail3(LBM_EINVAL, "null context");
    if (n < 0) return fail3(LBM_EINVAL, "negative step count");
    LBM3_HIP(hipSetDevice(ctx->device));
    const int64_t block = 2 * (int64_t)ctx->graph_k;
    if (ctx->graph_k > 0 && !ctx->graph_failed && n >= block) {
        if (ctx->graph && ctx->graph_cur != ctx->cur) drop_graph3(ctx); // captured from the other buffer
        if (!ctx->graph) build_graph3(ctx);
        if (ctx->graph) {
            while (n >= block) {
                LBM3_HIP(hipGraphLaunch(ctx->graph, ctx->stream));
                ctx->steps += block;
                n -= block;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        LBM3_HIP(lbm3::launch_step3(kprec(ctx->precision), ctx->args()));
        ctx->cur ^= 1;
        ++ctx->steps;
    }
    return LBM_OK;
}

lbm_status lbm3d_set_graph_steps(lbm3d_ctx *ctx, int32_t k)
{
    if (!ctx) return fail3(LBM_EINVAL, "null context");
    if (k < 0 || k > 4096) return fail3(LBM_EINVAL, "graph steps must lie in [0, 4096]");
    LBM3_HIP(hipSetDevice(ctx->device));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph3(ctx);
    ctx->graph_k = k;
    ctx->graph_failed = false;
    return LBM_OK;
}

int64_t lbm3d_steps_taken(const lbm3d_ctx *ctx) { return ctx ? ctx->steps : -1; }

lbm_status lbm3d_set_schedule(lbm3d_ctx *ctx, int32_t fused, int32_t tile_x, int32_t tile_y, int32_t z_chunk)
{
    if (!ctx) return fail3(LBM_EINVAL, "null context");
    if (fused != 0 && fused != 1) return fail3(LBM_EINVAL, "fused must be 0 or 1");
    if (fused) {
        if (!lbm3::fused3_shape_ok(tile_x, tile_y))
            return fail3(LBM_EINVAL, "fused tile must be 32 x 8, 32 x 16, 64 x 4, 64 x 8 or 64 x 16");
        if (z_chunk < 1) return fail3(LBM_EINVAL, "z_chunk must be >= 1");
        if (lbm3::fused3_blocks(ctx->grid.nx, ctx->grid.ny, ctx->grid.nz, tile_x, tile_y, z_chunk) * tile_x * tile_y >
            (int64_t)UINT32_MAX)
            return fail3(LBM_EINVAL, "z_chunk too small for this grid (launch above 2^32 threads)");
        ctx->tile_x = tile_x;
        ctx->tile_y = tile_y;
        ctx->zchunk = z_chunk;
    }
    ctx->fused = fused;
    LBM3_HIP(hipSetDevice(ctx->device));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph3(ctx); // the captured launches carry the schedule
    return LBM_OK;
}

// Checkpoint layout: a 64-byte header {magic, precision, nx, ny, nz, 0,
// steps, population bytes, FP32 base density, 16 reserved bytes}, then the
// raw population buffer of the current state, so that a restore continues
// bit for bit in either precision.
static const uint32_t kMagic3 = 0x334d424cu; // "LBM3"

static uint64_t state_pop_bytes3(const lbm3d_ctx *c)
{
    return 19 * (uint64_t)c->L.dstride * (c->precision == LBM_FP64 ? 8 : 4);
}

size_t lbm3d_state_bytes(const lbm3d_ctx *ctx) { return ctx ? 64 + state_pop_bytes3(ctx) : 0; }

lbm_status lbm3d_save_state(lbm3d_ctx *ctx, void *host_buf, size_t bytes)
{
    lbm::TraceRange trace_("lbm3d_save_state");
    if (!ctx || !host_buf) return fail3(LBM_EINVAL, "null argument");
    if (bytes < lbm3d_state_bytes(ctx)) return fail3(LBM_EINVAL, "buffer smaller than lbm3d_state_bytes()");
    LBM3_HIP(hipSetDevice(ctx->device));
    unsigned char *p = static_cast<unsigned char *>(host_buf);
    const uint64_t pb = state_pop_bytes3(ctx);
    const uint32_t h[6] = {kMagic3, (uint32_t)ctx->precision, (uint32_t)ctx->grid.nx, (uint32_t)ctx->grid.ny,
                           (uint32_t)ctx->grid.nz, 0u};
    std::memset(p, 0, 64);
    std::memcpy(p, h, 24);
    std::memcpy(p + 24, &ctx->steps, 8);
    std::memcpy(p + 32, &pb, 8);
    std::memcpy(p + 40, &ctx->run.r.pd.rho_ref, 8);
    LBM3_HIP(hipMemcpyAsync(p + 64, ctx->fbuf(ctx->cur), pb, hipMemcpyDeviceToHost, ctx->stream));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm3d_load_state(lbm3d_ctx *ctx, const void *host_buf, size_t bytes)
{
    lbm::TraceRange trace_("lbm3d_load_state");
    if (!ctx || !host_buf) return fail3(LBM_EINVAL, "null argument");
    if (bytes < 64) return fail3(LBM_EINVAL, "checkpoint too short");
    const unsigned char *p = static_cast<const unsigned char *>(host_buf);
    uint32_t h[6];
    int64_t steps;
    uint64_t pb;
    double ref;
    std::memcpy(h, p, 24);
    std::memcpy(&steps, p + 24, 8);
    std::memcpy(&pb, p + 32, 8);
    std::memcpy(&ref, p + 40, 8);
    if (h[0] != kMagic3 || h[1] != (uint32_t)ctx->precision || h[2] != (uint32_t)ctx->grid.nx ||
        h[3] != (uint32_t)ctx->grid.ny || h[4] != (uint32_t)ctx->grid.nz || pb != state_pop_bytes3(ctx) ||
        steps < 0 || !std::isfinite(ref))
        return fail3(LBM_ESTATE, "checkpoint does not match this context");
    if (bytes < 64 + pb) return fail3(LBM_EINVAL, "checkpoint truncated");
    LBM3_HIP(hipSetDevice(ctx->device));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    ctx->steps = steps;
    ctx->run.r.pd.rho_ref = ref;
    lbm_status s = upload_run3(ctx);
    if (s != LBM_OK) return s;
    LBM3_HIP(hipMemcpyAsync(ctx->fbuf(ctx->cur), p + 64, pb, hipMemcpyHostToDevice, ctx->stream));
    LBM3_HIP(hipMemsetAsync(ctx->dstatus(), 0, sizeof(int32_t), ctx->stream));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm3d_get_populations(lbm3d_ctx *ctx, double *f)
{
    lbm::TraceRange trace_("lbm3d_get_populations");
    if (!ctx || !f) return fail3(LBM_EINVAL, "null argument");
    LBM3_HIP(hipSetDevice(ctx->device));
    const int64_t N = ctx->nodes();
    LBM3_HIP(lbm3::launch_util3(kprec(ctx->precision), 0, ctx->drun(), ctx->fbuf(ctx->cur), nullptr, nullptr,
                                ctx->staging(), N, ctx->stream));
    LBM3_HIP(hipMemcpyAsync(f, ctx->staging(), sizeof(double) * 19 * N, hipMemcpyDeviceToHost, ctx->stream));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm3d_set_populations(lbm3d_ctx *ctx, const double *f)
{
    lbm::TraceRange trace_("lbm3d_set_populations");
    if (!ctx || !f) return fail3(LBM_EINVAL, "null argument");
    const int64_t N = ctx->nodes();
    for (int64_t i = 0; i < 19 * N; ++i)
        if (!std::isfinite(f[i])) return fail3(LBM_EINVAL, "populations must be finite");
    LBM3_HIP(hipSetDevice(ctx->device));
    LBM3_HIP(hipMemcpyAsync(ctx->staging(), f, sizeof(double) * 19 * N, hipMemcpyHostToDevice, ctx->stream));
    LBM3_HIP(lbm3::launch_util3(kprec(ctx->precision), 2, ctx->drun(), nullptr, ctx->fbuf(ctx->cur), nullptr,
                                ctx->staging(), N, ctx->stream));
    LBM3_HIP(hipMemsetAsync(ctx->dstatus(), 0, sizeof(int32_t), ctx->stream));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm3d_moments(lbm3d_ctx *ctx, double *rho, double *ux, double *uy, double *uz)
{
    lbm::TraceRange trace_("lbm3d_moments");
    if (!ctx || !rho) return fail3(LBM_EINVAL, "null argument");
    LBM3_HIP(hipSetDevice(ctx->device));
    const int64_t N = ctx->nodes();
    lbm_status s = psi_refresh(ctx);
    if (s != LBM_OK) return s;
    double *st = ctx->staging();
    LBM3_HIP(lbm3::launch_util3(kprec(ctx->precision), 1, ctx->drun(), ctx->fbuf(ctx->cur), nullptr,
                                ctx->ws + ctx->L.psi, st, N, ctx->stream));
    LBM3_HIP(hipMemcpyAsync(rho, st, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
    double *u[3] = {ux, uy, uz};
    for (int i = 0; i < 3; ++i)
        if (u[i]) LBM3_HIP(hipMemcpyAsync(u[i], st + (i + 1) * N, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
    int32_t stat = 0;
    LBM3_HIP(hipMemcpyAsync(&stat, ctx->dstatus(), sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    return stat ? fail3(LBM_EDIVERGED, "the run has diverged") : LBM_OK;
}

lbm_status lbm3d_diagnostics(lbm3d_ctx *ctx, int32_t dims, double cx, double cy, double cz, double r_in,
                             double r_out, lbm_diag *out)
{
    lbm::TraceRange trace_("lbm3d_diagnostics");
    if (!ctx || !out) return fail3(LBM_EINVAL, "null argument");
    if (dims != 2 && dims != 3) return fail3(LBM_EINVAL, "dims must be 2 (cylinder) or 3 (sphere)");
    for (double v : {cx, cy, cz, r_in, r_out})
        if (!std::isfinite(v)) return fail3(LBM_EINVAL, "diagnostic region must be finite");
    LBM3_HIP(hipSetDevice(ctx->device));
    lbm_status s = psi_refresh(ctx);
    if (s != LBM_OK) return s;
    double *partial = reinterpret_cast<double *>(ctx->ws + ctx->L.partial);
    LBM3_HIP(lbm3::launch_diag3(kprec(ctx->precision), ctx->drun(), ctx->fbuf(ctx->cur), ctx->ws + ctx->L.psi, dims,
                                cx, cy, cz, r_in, r_out, partial, ctx->nodes(), ctx->stream));
    std::vector<double> h(8 * (size_t)ctx->L.nblocks);
    int32_t stat = 0;
    LBM3_HIP(hipMemcpyAsync(h.data(), partial, sizeof(double) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
    LBM3_HIP(hipMemcpyAsync(&stat, ctx->dstatus(), sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    LBM3_HIP(hipStreamSynchronize(ctx->stream));
    // fixed-order FP64 reduction of the block partials
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = 0; b < ctx->L.nblocks; ++b) {
        for (int q = 0; q < 7; ++q) v[q] += h[8 * b + q];
        v[7] = std::fmax(v[7], h[8 * b + 7]);
    }
    const double N = (double)ctx->nodes();
    out->mass = v[0];
    out->rho_in = v[2] > 0 ? v[1] / v[2] : NAN;
    out->rho_out = v[4] > 0 ? v[3] / v[4] : NAN;
    out->p_in = v[2] > 0 ? v[5] / v[2] : NAN;
    out->p_out = v[4] > 0 ? v[6] / v[4] : NAN;
    out->dp = out->p_in - out->p_out;
    const double excess = out->mass - out->rho_out * N, drho = out->rho_in - out->rho_out;
    out->r_eq = dims == 3 ? std::cbrt(3.0 * excess / (4.0 * M_PI * drho))
                          : std::sqrt(excess / (M_PI * ctx->grid.nz * drho));
    out->max_speed = v[7];
    out->status = stat;
    out->reserved = 0;
    return stat ? fail3(LBM_EDIVERGED, "the run has diverged") : LBM_OK;
}

// Times `steps` steps of each candidate schedule on the context's own state
// (which advances) and keeps the fastest.
lbm_status lbm3d_autotune(lbm3d_ctx *ctx, int32_t steps, int32_t *fused, int32_t *tile_x, int32_t *tile_y,
                          int32_t *z_chunk)
{
    lbm::TraceRange trace_("lbm3d_autotune");
    if (!ctx) return fail3(LBM_EINVAL, "null context");
    if (steps < 1) return fail3(LBM_EINVAL, "autotune needs at least 1 step per candidate");
    LBM3_HIP(hipSetDevice(ctx->device));
    struct Cand {
        int fused, tx, ty, zc;
    };
    const Cand cands[] = {{1, 64, 8, 64}, {1, 64, 8, 128}, {1, 64, 8, 32}, {1, 64, 4, 64}, {1, 32, 8, 64},
                          {1, 32, 16, 64}, {1, 64, 16, 64}, {0, 64, 8, 64}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LBM3_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail3(LBM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(he));
    }
    const Cand keep = {ctx->fused, ctx->tile_x, ctx->tile_y, ctx->zchunk};
    Cand pick = keep;
    float best = 0.f;
    lbm_status rc = LBM_OK;
    for (const Cand &c : cands) {
        // candidates that do not fit this grid's launch limits are skipped
        if (lbm3d_set_schedule(ctx, c.fused, c.tx, c.ty, c.zc) != LBM_OK) continue;
        if ((rc = lbm3d_step(ctx, 1)) != LBM_OK) break; // warm-up
        he = hipEventRecord(e0, ctx->stream);
        if (he == hipSuccess && (rc = lbm3d_step(ctx, steps)) != LBM_OK) break;
        if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            rc = fail3(LBM_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(he));
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
        (void)lbm3d_set_schedule(ctx, keep.fused, keep.tx, keep.ty, keep.zc);
        return rc;
    }
    if ((rc = lbm3d_set_schedule(ctx, pick.fused, pick.tx, pick.ty, pick.zc)) != LBM_OK) return rc;
    if (fused) *fused = pick.fused;
    if (tile_x) *tile_x = pick.tx;
    if (tile_y) *tile_y = pick.ty;
    if (z_chunk) *z_chunk = pick.zc;
    return LBM_OK;
}

lbm_status lbm3d_time_kernels(lbm3d_ctx *ctx, int64_t n, double *psi_ms, double *collide_ms)
{
    lbm::TraceRange trace_("lbm3d_time_kernels");
    if (!ctx || n < 1 || !psi_ms || !collide_ms) return fail3(LBM_EINVAL, "need n >= 1 and two outputs");
    LBM3_HIP(hipSetDevice(ctx->device));
    std::vector<hipEvent_t> ev(4 * n, nullptr);
    lbm_status rc = LBM_OK;
    int64_t made = 0;
    for (; made < 4 * n; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) {
            rc = fail3(LBM_EDEVICE, "hipEventCreate failed");
            break;
        }
    double tp = 0.0, tc = 0.0;
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < n && rc == LBM_OK && e == hipSuccess; ++i) {
        lbm3::Step3Args a = ctx->args();
        a.ev_psi0 = ev[4 * i];
        a.ev_psi1 = ev[4 * i + 1];
        a.ev_col0 = ev[4 * i + 2];
        a.ev_col1 = ev[4 * i + 3];
        e = lbm3::launch_step3(kprec(ctx->precision), a);
        if (e == hipSuccess) {
            ctx->cur ^= 1;
            ++ctx->steps;
        }
    }
    if (rc == LBM_OK && e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    for (int64_t i = 0; i < n && rc == LBM_OK && e == hipSuccess; ++i) {
        float a1 = 0.f, a2 = 0.f;
        if (!ctx->fused) e = hipEventElapsedTime(&a1, ev[4 * i], ev[4 * i + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&a2, ev[4 * i + 2], ev[4 * i + 3]);
        tp += a1;
        tc += a2;
    }
    if (rc == LBM_OK && e != hipSuccess) rc = fail3(LBM_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
    for (int64_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (rc == LBM_OK) {
        *psi_ms = tp / n;
        *collide_ms = tc / n;
    }
    return rc;
}

} // extern "C"
