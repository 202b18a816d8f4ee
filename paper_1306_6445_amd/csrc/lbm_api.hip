// Host runtime behind the C ABI of include/lbm.h: parameter validation,
// workspace layout, the tile work list, step scheduling (HIP graphs of 2k
// steps on the caller's stream) and the FP64 read-back paths.
#include "../../include/lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm_device.hpp"
#include "lbm_error.hpp"
#include "lbm_trace.hpp"
#include "lbm_kernels.hpp"

namespace {

thread_local std::string g_error;

lbm_status fail(lbm_status s, const std::string &msg)
{
    g_error = msg;
    return s;
}

#define LBM_HIP(call)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail(LBM_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t pop_bytes(int prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2); }
size_t psi_bytes(int prec) { return prec == LBM_FP64 ? 8 : 4; }

bool is_finite(double v) { return std::isfinite(v); }

const int kTileX[] = {32, 64, 128, 256};
const int kTileY[] = {1, 2, 4, 8};

bool tile_allowed(int tx, int ty)
{
    bool okx = false, oky = false;
    for (int v : kTileX) okx |= v == tx;
    for (int v : kTileY) oky |= v == ty;
    return okx && oky && tx * ty >= 64 && tx * ty <= lbm::kMaxTileThreads;
}

int64_t tiles_of(const lbm_grid &g, int tx, int ty)
{
    return (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
}

// Row stride of a run's device arrays (every kernel addresses rows by it).
// Dense rows: padding each row to 128 bytes of storage aligns the even
// steps' accesses, but on grids 64-512 nodes wide the padded line ends cost
// as much traffic as the alignment saves (FP32 +2%, FP64 -3.5%, bf16 -1% on
// the 512-run ensemble), so the rows stay unpadded.
int pitch_of(int nx, int /*prec*/) { return nx; }

// Elements from one direction's population array to the next: the run's
// nodes rounded up to 256 bytes, plus a skew of 17 x 256 bytes, so that the
// nine arrays of a grid whose size is a large power of two do not start at
// the same offset modulo the HBM channel interleave (a 4096 x 2048 FP32 grid
// streams about 10% faster with the skew).  The skew is never read.
constexpr size_t kDirSkewBytes = 17 * 256;
int64_t dstride_of(int64_t nodes, int prec)
{
    const size_t s = prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2);
    const size_t bytes = ((nodes * s + 255) & ~size_t(255)) + kDirSkewBytes;
    return (int64_t)(bytes / s);
}

struct Layout {
    size_t f = 0, f2 = 0, psi = 0, r0 = 0, r1 = 0, seed = 0, runs = 0, tiles = 0, ftiles = 0, status = 0,
           partial = 0, dout = 0, regions = 0, staging = 0;
    size_t total = 0;
    int64_t max_tiles = 0;
    int64_t pop_elems = 0;   // population elements of all runs, 9 x dstride each
    int64_t total_nodes = 0; // nodes of all runs including the row padding (pitch x ny each)
    int64_t max_nodes = 0;   // the same for the largest run (sizes the host staging area)
};

Layout make_layout(int nruns, const lbm_run_desc *runs, int prec)
{
    Layout L;
    for (int i = 0; i < nruns; ++i) {
        const int64_t n = (int64_t)pitch_of(runs[i].grid.nx, prec) * runs[i].grid.ny;
        L.total_nodes += n;
        L.pop_elems += 9 * dstride_of(n, prec);
        L.max_nodes = std::max(L.max_nodes, n);
    }
    for (int tx : kTileX)
        for (int ty : kTileY) {
            if (!tile_allowed(tx, ty)) continue;
            int64_t t = 0;
            for (int i = 0; i < nruns; ++i) t += tiles_of(runs[i].grid, tx, ty);
            L.max_tiles = std::max(L.max_tiles, t);
        }
    size_t off = 0;
    L.f = off;
    off = align256(off + pop_bytes(prec) * (size_t)L.pop_elems);
    // second population buffer: the fused schedule writes each step's state
    // to the buffer it did not read
    L.f2 = off;
    off = align256(off + pop_bytes(prec) * (size_t)L.pop_elems);
    L.psi = off;
    off = align256(off + psi_bytes(prec) * (size_t)L.total_nodes);
    // writer densities of bf16 storage, one FP32 array per step parity
    const size_t rbytes = prec == LBM_FP32_BF16STORE ? sizeof(float) * (size_t)L.total_nodes : 0;
    L.r0 = off;
    off = align256(off + rbytes);
    L.r1 = off;
    off = align256(off + rbytes);
    L.seed = off;
    off = align256(off + 2 * sizeof(uint32_t));
    L.runs = off;
    off = align256(off + sizeof(lbm::RunDev) * nruns);
    L.tiles = off;
    off = align256(off + sizeof(lbm::Tile) * (size_t)L.max_tiles);
    L.ftiles = off; // tiles of tx x (R ty) nodes: never more than of tx x ty
    off = align256(off + sizeof(lbm::Tile) * (size_t)L.max_tiles);
    L.status = off;
    off = align256(off + sizeof(int32_t) * nruns);
    L.partial = off;
    off = align256(off + 8 * sizeof(double) * (size_t)L.max_tiles);
    L.dout = off;
    off = align256(off + 8 * sizeof(double) * nruns);
    L.regions = off;
    off = align256(off + 4 * sizeof(double) * nruns);
    L.staging = off;
    off = align256(off + 9 * sizeof(double) * (size_t)L.max_nodes);
    L.total = off;
    return L;
}

lbm_status validate_run(const lbm_run_desc *r)
{
    if (!r) return fail(LBM_EINVAL, "null run descriptor");
    const lbm_grid &g = r->grid;
    if (g.nx < 1 || g.ny < 1) return fail(LBM_EINVAL, "nx and ny must be >= 1");
    if ((int64_t)g.nx * g.ny > (int64_t)1 << 31) return fail(LBM_EINVAL, "grid too large for one run");
    for (int bc : {g.bc_x, g.bc_y})
        if (bc != LBM_BC_PERIODIC && bc != LBM_BC_BOUNCEBACK) return fail(LBM_EINVAL, "unknown boundary kind");
    const lbm_rates &s = r->rates;
    for (double v : {s.s_rho, s.s_e, s.s_zeta, s.s_j, s.s_q, s.s_nu})
        if (!(v > 0.0 && v < 2.0)) return fail(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
    if (!(r->kappa >= 0.0 && r->kappa < 1.0)) return fail(LBM_EINVAL, "kappa must lie in [0, 1)");
    if (!is_finite(r->epsilon) || r->epsilon < 0.0) return fail(LBM_EINVAL, "epsilon must be finite and >= 0");
    if (r->epsilon != 0.0 && s.s_zeta != s.s_e)
        return fail(LBM_EINVAL, "epsilon != 0 requires s_zeta == s_e (Eq. 8)");
    if (!is_finite(r->G)) return fail(LBM_EINVAL, "G must be finite");
    for (double v : r->eos.p)
        if (!is_finite(v)) return fail(LBM_EINVAL, "EOS parameters must be finite");
    const double *p = r->eos.p;
    switch (r->eos.kind) {
    case LBM_EOS_CS:
        if (!(p[0] > 0 && p[1] > 0 && p[2] > 0 && p[3] > 0))
            return fail(LBM_EINVAL, "Carnahan-Starling a, b, R, T must be > 0");
        if (!(r->G < 0.0)) return fail(LBM_EINVAL, "the sqrt pseudopotential needs G < 0");
        break;
    case LBM_EOS_PIECEWISE:
        if (!(p[3] > 0 && p[3] < p[4])) return fail(LBM_EINVAL, "piecewise EOS needs 0 < rho1 < rho2");
        if (!(r->G < 0.0)) return fail(LBM_EINVAL, "the sqrt pseudopotential needs G < 0");
        break;
    case LBM_EOS_SC_EXP:
        if (!(p[0] > 0 && p[1] > 0)) return fail(LBM_EINVAL, "psi0 and rho0 must be > 0");
        if (r->epsilon != 0.0 && r->G == 0.0) return fail(LBM_EINVAL, "epsilon != 0 needs G != 0");
        break;
    default:
        return fail(LBM_EINVAL, "unknown EOS kind");
    }
    return LBM_OK;
}

bool valid_precision(int p) { return p == LBM_FP64 || p == LBM_FP32 || p == LBM_FP32_BF16STORE; }

int kernel_precision(int p) { return p == LBM_FP64 ? lbm::PREC_FP64 : (p == LBM_FP32 ? lbm::PREC_FP32 : lbm::PREC_BF16); }

} // namespace

struct lbm_ctx {
    int device = 0;
    int precision = LBM_FP64;
    int nruns = 0;
    std::vector<lbm_run_desc> desc;
    std::vector<lbm::RunDev> rdev;
    std::vector<int> ref_set;       // FP32: 1 once lbm_run_set_reference_density chose the run's base
    std::vector<lbm::Tile> tiles;   // tx x ty tiles of every run (two-kernel step and diagnostics)
    std::vector<lbm::Tile> ftiles;  // tx x (fused ty) tiles of every run (fused step)
    Layout L;
    unsigned char *ws = nullptr;
    bool own_ws = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int tx = 64, ty = 4;
    int64_t steps = 0;
    int graph_k = 16;
    int xcd = 1;
    int fused = 0;         // nodes per thread of the fused kernel (1, 2, 4); 0: psi + collide in place
                           // (2 at creation)
    int halo = 1;          // psi halo of the collide tile: 2 once a run uses the multi-range force
    int cur = 0;           // population buffer holding the current state (0: L.f, 1: L.f2)
    int graph_cur = 0;     // buffer the captured graph starts from
    hipGraphExec_t graph = nullptr;
    bool graph_failed = false;

    template <typename T> T *at(size_t off) { return reinterpret_cast<T *>(ws + off); }
    unsigned char *fbuf(int k) { return ws + (k ? L.f2 : L.f); }

    lbm::StepArgs step_args()
    {
        lbm::StepArgs a;
        a.runs = at<lbm::RunDev>(L.runs);
        a.tiles = at<lbm::Tile>(L.tiles);
        a.ntiles = (int)tiles.size();
        a.tx = tx;
        a.ty = ty;
        a.f = fbuf(cur);
        a.f_alt = fbuf(cur ^ 1);
        a.psi = ws + L.psi;
        a.status = at<int32_t>(L.status);
        a.stream = stream;
        a.xcd = xcd;
        a.fused = fused;
        a.ftiles = at<lbm::Tile>(L.ftiles);
        a.nftiles = (int)ftiles.size();
        if (precision == LBM_FP32_BF16STORE) {
            a.r0 = at<float>(L.r0);
            a.r1 = at<float>(L.r1);
        }
        a.seed = at<uint32_t>(L.seed);
        a.halo = halo;
        return a;
    }

    int parity() const { return (int)(steps & 1); }
};

namespace {

// Work lists: tiles of every run in row-major order, runs one after another.
void build_tiles(lbm_ctx *c)
{
    c->tiles.clear();
    c->ftiles.clear();
    const int fty = c->ty * std::max(c->fused, 1);
    for (int r = 0; r < c->nruns; ++r) {
        const lbm_grid &g = c->desc[r].grid;
        c->rdev[r].tile_begin = (int32_t)c->tiles.size();
        for (int y0 = 0; y0 < g.ny; y0 += c->ty)
            for (int x0 = 0; x0 < g.nx; x0 += c->tx) c->tiles.push_back(lbm::Tile{r, x0, y0, 0});
        c->rdev[r].tile_count = (int32_t)c->tiles.size() - c->rdev[r].tile_begin;
        for (int y0 = 0; y0 < g.ny; y0 += fty)
            for (int x0 = 0; x0 < g.nx; x0 += c->tx) c->ftiles.push_back(lbm::Tile{r, x0, y0, 0});
    }
}

lbm_status upload_tables(lbm_ctx *c)
{
    LBM_HIP(hipSetDevice(c->device));
    LBM_HIP(hipMemcpyAsync(c->ws + c->L.runs, c->rdev.data(), sizeof(lbm::RunDev) * c->nruns,
                           hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipMemcpyAsync(c->ws + c->L.tiles, c->tiles.data(), sizeof(lbm::Tile) * c->tiles.size(),
                           hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipMemcpyAsync(c->ws + c->L.ftiles, c->ftiles.data(), sizeof(lbm::Tile) * c->ftiles.size(),
                           hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Finishes one run's record (derived and FP32 constants) and enqueues its
// upload on the context's stream (kernels read the table at launch).
lbm_status upload_run(lbm_ctx *c, int run)
{
    lbm::finish_rundev(c->rdev[run]);
    LBM_HIP(hipMemcpyAsync(c->ws + c->L.runs + sizeof(lbm::RunDev) * run, &c->rdev[run], sizeof(lbm::RunDev),
                           hipMemcpyHostToDevice, c->stream));
    return LBM_OK;
}

void drop_graph(lbm_ctx *c)
{
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

lbm::RunDev make_rundev(const lbm_run_desc &d)
{
    lbm::RunDev r;
    std::memset(&r, 0, sizeof(r));
    r.nx = d.grid.nx;
    r.ny = d.grid.ny;
    r.bc_x = d.grid.bc_x;
    r.bc_y = d.grid.bc_y;
    r.eos_kind = d.eos.kind;
    lbm::RunPar<double> &k = r.pd;
    for (int i = 0; i < 6; ++i) k.eos[i] = d.eos.p[i];
    k.G = d.G;
    k.G2 = 0.0;
    k.G_eos = d.G;
    k.kappa = d.kappa;
    // Eq. (8) constant sigma = -epsilon / (16 G); the moment-space term is
    // 12 sigma |F|^2 / (psi^2 (tau_e - 1/2)) with tau_e = 1 / s_e.
    const double sigma = d.epsilon == 0.0 ? 0.0 : -d.epsilon / (16.0 * d.G);
    k.sig_coef = 12.0 * sigma / (1.0 / d.rates.s_e - 0.5);
    k.s_e = d.rates.s_e;
    k.s_zeta = d.rates.s_zeta;
    k.s_q = d.rates.s_q;
    k.s_nu = d.rates.s_nu;
    k.rho_ref = 0.0;
    lbm::finish_rundev(r);
    return r;
}

lbm_status check_ctx(const lbm_ctx *c)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    return LBM_OK;
}

lbm_status check_run(const lbm_ctx *c, int32_t run)
{
    if (!c) return fail(LBM_EINVAL, "null context");
    if (run < 0 || run >= c->nruns) return fail(LBM_EINVAL, "run index out of range");
    return LBM_OK;
}

int64_t run_nodes(const lbm_ctx *c, int run) { return (int64_t)c->desc[run].grid.nx * c->desc[run].grid.ny; }

lbm_status util(lbm_ctx *c, int op, int run, double *buf, const double *ux = nullptr, const double *uy = nullptr)
{
    lbm::UtilArgs u;
    u.op = op;
    u.runs = c->at<lbm::RunDev>(c->L.runs);
    u.run = run;
    u.nodes = run_nodes(c, run);
    u.f = c->fbuf(c->cur);
    u.psi = c->ws + c->L.psi;
    u.buf = buf;
    u.ux = ux;
    u.uy = uy;
    u.parity = c->parity();
    u.stream = c->stream;
    if (c->precision == LBM_FP32_BF16STORE) {
        u.r0 = c->at<float>(c->L.r0);
        u.r1 = c->at<float>(c->L.r1);
    }
    LBM_HIP(lbm::launch_util(kernel_precision(c->precision), u));
    return LBM_OK;
}

// Rounding-seed counters of bf16 storage: a step of parity p writes slot p as
// slot (p ^ 1) + 1; starting from {0, 2^32 - 1} the seed of step t is t.
lbm_status reset_seed(lbm_ctx *c, int64_t steps)
{
    const uint32_t v[2] = {(uint32_t)steps, (uint32_t)(steps - 1)};
    uint32_t w[2];
    w[steps & 1] = v[0];       // not read before it is rewritten
    w[(steps & 1) ^ 1] = v[1]; // the last step's seed
    LBM_HIP(hipMemcpyAsync(c->ws + c->L.seed, w, sizeof(w), hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status refresh_psi(lbm_ctx *c)
{
    LBM_HIP(lbm::launch_psi(kernel_precision(c->precision), c->step_args(), c->parity()));
    return LBM_OK;
}

lbm_status read_status(lbm_ctx *c, std::vector<int32_t> &st)
{
    st.assign(c->nruns, 0);
    LBM_HIP(hipMemcpyAsync(st.data(), c->ws + c->L.status, sizeof(int32_t) * c->nruns, hipMemcpyDeviceToHost,
                           c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// After a fused step the state lives in the other buffer.
void swap_buffers(lbm_ctx *c, lbm::StepArgs &a)
{
    std::swap(a.f, a.f_alt);
    c->cur ^= 1;
}

lbm_status step_eager(lbm_ctx *c, int64_t n)
{
    const int prec = kernel_precision(c->precision);
    lbm::StepArgs a = c->step_args();
    for (int64_t i = 0; i < n; ++i) {
        LBM_HIP(lbm::launch_step(prec, a, c->parity()));
        ++c->steps;
        if (c->fused) swap_buffers(c, a);
    }
    return LBM_OK;
}

lbm_status build_graph(lbm_ctx *c)
{
    const int prec = kernel_precision(c->precision);
    lbm::StepArgs a = c->step_args();
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        c->graph_failed = true;
        return LBM_OK;
    }
    // 2k steps from an even step count; fused steps alternate the buffers
    // and end on the one they started from
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 * c->graph_k && e == hipSuccess; ++i) {
        e = lbm::launch_step(prec, a, i & 1);
        if (c->fused) std::swap(a.f, a.f_alt);
    }
    c->graph_cur = c->cur;
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->graph_failed = true;
        return LBM_OK;
    }
    hipError_t e3 = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        c->graph = nullptr;
        (void)hipGetLastError();
        c->graph_failed = true;
    }
    return LBM_OK;
}

lbm_status create_impl(int32_t nruns, const lbm_run_desc *runs, int32_t precision, void *workspace,
                       size_t workspace_bytes, void *stream, lbm_ctx **out)
{
    if (!out) return fail(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (nruns < 1 || !runs) return fail(LBM_EINVAL, "need at least one run");
    if (!valid_precision(precision)) return fail(LBM_EINVAL, "unknown precision");
    for (int i = 0; i < nruns; ++i) {
        lbm_status s = validate_run(&runs[i]);
        if (s != LBM_OK) return fail(s, "run " + std::to_string(i) + ": " + g_error);
    }
    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_ENOMEM, "host allocation failed");
    c->precision = precision;
    c->nruns = nruns;
    // default schedule: the fused kernel, two nodes per thread (faster on
    // MI355X than two kernels for every storage precision)
    c->fused = 2;
    c->desc.assign(runs, runs + nruns);
    c->L = make_layout(nruns, runs, precision);
    if (workspace && workspace_bytes < c->L.total) {
        delete c;
        return fail(LBM_ENOMEM, "workspace smaller than lbm_workspace_bytes()");
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
        delete c;
        return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    }
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return fail(LBM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    if (stream) {
        c->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return fail(LBM_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        c->own_stream = true;
    }
    if (workspace) {
        c->ws = static_cast<unsigned char *>(workspace);
    } else {
        e = hipMalloc(&c->ws, c->L.total);
        if (e != hipSuccess) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(LBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        c->own_ws = true;
    }
    int64_t foff = 0, noff = 0;
    c->rdev.resize(nruns);
    c->ref_set.assign(nruns, 0);
    for (int i = 0; i < nruns; ++i) {
        c->rdev[i] = make_rundev(runs[i]);
        c->rdev[i].pitch = pitch_of(runs[i].grid.nx, precision);
        const int64_t n = (int64_t)c->rdev[i].pitch * runs[i].grid.ny;
        c->rdev[i].dstride = dstride_of(n, precision);
        c->rdev[i].f_off = foff;
        c->rdev[i].n_off = noff;
        foff += 9 * c->rdev[i].dstride;
        noff += n;
    }
    build_tiles(c);
    lbm_status s = upload_tables(c);
    if (s == LBM_OK) {
        hipError_t e2 = hipMemsetAsync(c->ws + c->L.status, 0, sizeof(int32_t) * nruns, c->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
        if (e2 != hipSuccess) s = fail(LBM_EDEVICE, std::string("status clear: ") + hipGetErrorString(e2));
    }
    if (s == LBM_OK) s = reset_seed(c, 0);
    if (s != LBM_OK) {
        lbm_destroy(c);
        return s;
    }
    *out = c;
    return LBM_OK;
}

} // namespace

extern "C" {

const char *lbm_last_error(void) { return g_error.c_str(); }

lbm_status lbm_validate_run(const lbm_run_desc *run) { return validate_run(run); }

lbm_status lbm_validate(const lbm_grid *grid, const lbm_eos *eos, double G, const lbm_rates *rates, double kappa,
                        double epsilon)
{
    if (!grid || !eos || !rates) return fail(LBM_EINVAL, "null argument");
    lbm_run_desc d;
    d.grid = *grid;
    d.eos = *eos;
    d.G = G;
    d.rates = *rates;
    d.kappa = kappa;
    d.epsilon = epsilon;
    return validate_run(&d);
}

size_t lbm_batch_workspace_bytes(int32_t nruns, const lbm_run_desc *runs, int32_t precision)
{
    if (nruns < 1 || !runs || !valid_precision(precision)) return 0;
    for (int i = 0; i < nruns; ++i)
        if (runs[i].grid.nx < 1 || runs[i].grid.ny < 1) return 0;
    return make_layout(nruns, runs, precision).total;
}

size_t lbm_workspace_bytes(const lbm_grid *grid, int32_t precision)
{
    if (!grid) return 0;
    lbm_run_desc d;
    std::memset(&d, 0, sizeof(d));
    d.grid = *grid;
    return lbm_batch_workspace_bytes(1, &d, precision);
}

lbm_status lbm_batch_create(int32_t nruns, const lbm_run_desc *runs, int32_t precision, void *workspace,
                            size_t workspace_bytes, void *stream, lbm_ctx **out)
{
    return create_impl(nruns, runs, precision, workspace, workspace_bytes, stream, out);
}

lbm_status lbm_create(const lbm_grid *grid, const lbm_eos *eos, double G, const lbm_rates *rates, double kappa,
                      double epsilon, int32_t precision, void *workspace, size_t workspace_bytes, void *stream,
                      lbm_ctx **out)
{
    if (!grid || !eos || !rates) return fail(LBM_EINVAL, "null argument");
    lbm_run_desc d;
    d.grid = *grid;
    d.eos = *eos;
    d.G = G;
    d.rates = *rates;
    d.kappa = kappa;
    d.epsilon = epsilon;
    return create_impl(1, &d, precision, workspace, workspace_bytes, stream, out);
}

int32_t lbm_num_runs(const lbm_ctx *ctx) { return ctx ? ctx->nruns : 0; }

int64_t lbm_steps_taken(const lbm_ctx *ctx) { return ctx ? ctx->steps : -1; }

void lbm_destroy(lbm_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

lbm_status lbm_run_init_density(lbm_ctx *ctx, int32_t run, const double *rho, const double *ux, const double *uy)
{
    lbm::TraceRange trace_("lbm_run_init_density");
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!rho) return fail(LBM_EINVAL, "null density");
    const int64_t N = run_nodes(ctx, run);
    double rmin = HUGE_VAL, rmax = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        if (!(rho[i] > 0.0) || !is_finite(rho[i])) return fail(LBM_EINVAL, "density must be finite and > 0");
        rmin = std::min(rmin, rho[i]);
        rmax = std::max(rmax, rho[i]);
        if ((ux && !is_finite(ux[i])) || (uy && !is_finite(uy[i]))) return fail(LBM_EINVAL, "velocity must be finite");
    }
    LBM_HIP(hipSetDevice(ctx->device));
    // Base density of the FP32 deviation storage: the lighter phase, i.e. the
    // smallest initial density, unless lbm_run_set_reference_density chose
    // one (kept).  FP64 stores the populations themselves; bf16 takes each
    // population's writer density (the initial density of its upwind node
    // here), not a per-run constant.
    (void)rmax;
    if (ctx->precision == LBM_FP32 && !ctx->ref_set[run]) ctx->rdev[run].pd.rho_ref = rmin;
    if ((s = upload_run(ctx, run)) != LBM_OK) return s;
    double *st = ctx->at<double>(ctx->L.staging);
    LBM_HIP(hipMemcpyAsync(st, rho, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    if (ux) LBM_HIP(hipMemcpyAsync(st + N, ux, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    if (uy) LBM_HIP(hipMemcpyAsync(st + 2 * N, uy, sizeof(double) * N, hipMemcpyHostToDevice, ctx->stream));
    s = util(ctx, lbm::UTIL_INIT, run, st, ux ? st + N : nullptr, uy ? st + 2 * N : nullptr);
    if (s != LBM_OK) return s;
    LBM_HIP(hipMemsetAsync(ctx->ws + ctx->L.status + sizeof(int32_t) * run, 0, sizeof(int32_t), ctx->stream));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_init_density(lbm_ctx *ctx, const double *rho, const double *ux, const double *uy)
{
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    ctx->steps = 0;
    if (ctx->precision == LBM_FP32_BF16STORE) {
        LBM_HIP(hipSetDevice(ctx->device));
        if ((s = reset_seed(ctx, 0)) != LBM_OK) return s;
    }
    return lbm_run_init_density(ctx, 0, rho, ux, uy);
}

lbm_status lbm_step(lbm_ctx *ctx, int64_t n)
{
    lbm::TraceRange trace_("lbm_step");
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (n < 0) return fail(LBM_EINVAL, "negative step count");
    if (n == 0) return LBM_OK;
    LBM_HIP(hipSetDevice(ctx->device));
    const int64_t block = 2 * (int64_t)ctx->graph_k;
    if (ctx->graph_k > 0 && !ctx->graph_failed && n >= block + ctx->parity()) {
        if (ctx->parity()) {
            s = step_eager(ctx, 1);
            --n;
            if (s != LBM_OK) return s;
        }
        if (ctx->graph && ctx->graph_cur != ctx->cur) drop_graph(ctx); // captured from the other buffer
        if (!ctx->graph) {
            s = build_graph(ctx);
            if (s != LBM_OK) return s;
        }
        if (ctx->graph) {
            while (n >= block) {
                LBM_HIP(hipGraphLaunch(ctx->graph, ctx->stream));
                ctx->steps += block;
                n -= block;
            }
        }
    }
    return step_eager(ctx, n);
}

lbm_status lbm_run_moments(lbm_ctx *ctx, int32_t run, double *rho, double *ux, double *uy)
{
    lbm::TraceRange trace_("lbm_run_moments");
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!rho) return fail(LBM_EINVAL, "null density output");
    LBM_HIP(hipSetDevice(ctx->device));
    const int64_t N = run_nodes(ctx, run);
    double *st = ctx->at<double>(ctx->L.staging);
    if ((s = refresh_psi(ctx)) != LBM_OK) return s;
    if ((s = util(ctx, lbm::UTIL_MOMENTS, run, st)) != LBM_OK) return s;
    LBM_HIP(hipMemcpyAsync(rho, st, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
    if (ux) LBM_HIP(hipMemcpyAsync(ux, st + N, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
    if (uy) LBM_HIP(hipMemcpyAsync(uy, st + 2 * N, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
    std::vector<int32_t> stt;
    if ((s = read_status(ctx, stt)) != LBM_OK) return s;
    return stt[run] ? fail(LBM_EDIVERGED, "run " + std::to_string(run) + " has diverged") : LBM_OK;
}

lbm_status lbm_run_density_column(lbm_ctx *ctx, int32_t run, int32_t x, double *rho)
{
    lbm::TraceRange trace_("lbm_run_density_column");
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!rho) return fail(LBM_EINVAL, "null output");
    if (x < 0 || x >= ctx->desc[run].grid.nx) return fail(LBM_EINVAL, "column index out of range");
    LBM_HIP(hipSetDevice(ctx->device));
    const int ny = ctx->desc[run].grid.ny;
    double *st = ctx->at<double>(ctx->L.staging);
    lbm::UtilArgs u;
    u.op = lbm::UTIL_COLUMN;
    u.runs = ctx->at<lbm::RunDev>(ctx->L.runs);
    u.run = run;
    u.nodes = ny;
    u.f = ctx->fbuf(ctx->cur);
    u.psi = nullptr;
    u.buf = st;
    u.ux = u.uy = nullptr;
    u.parity = ctx->parity();
    u.index = x;
    u.stream = ctx->stream;
    if (ctx->precision == LBM_FP32_BF16STORE) {
        u.r0 = ctx->at<float>(ctx->L.r0);
        u.r1 = ctx->at<float>(ctx->L.r1);
    }
    LBM_HIP(lbm::launch_util(kernel_precision(ctx->precision), u));
    LBM_HIP(hipMemcpyAsync(rho, st, sizeof(double) * ny, hipMemcpyDeviceToHost, ctx->stream));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx *ctx, double *rho, double *ux, double *uy)
{
    return lbm_run_moments(ctx, 0, rho, ux, uy);
}

lbm_status lbm_run_get_window(lbm_ctx *ctx, int32_t run, int32_t x0, int32_t y0, int32_t w, int32_t h, double *f)
{
    lbm::TraceRange trace_("lbm_run_get_window");
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!f) return fail(LBM_EINVAL, "null output");
    const lbm_grid &g = ctx->desc[run].grid;
    if (w < 1 || h < 1 || w > g.nx || h > g.ny) return fail(LBM_EINVAL, "window size must lie in [1, nx] x [1, ny]");
    if ((g.bc_x == LBM_BC_BOUNCEBACK && (x0 < 0 || x0 + w > g.nx)) ||
        (g.bc_y == LBM_BC_BOUNCEBACK && (y0 < 0 || y0 + h > g.ny)))
        return fail(LBM_EINVAL, "window leaves the grid across a wall");
    if ((int64_t)9 * w * h > (int64_t)9 * run_nodes(ctx, run)) return fail(LBM_EINVAL, "window too large");
    LBM_HIP(hipSetDevice(ctx->device));
    // the staging area holds 9 x (largest run) doubles; a window is at most one run
    double *st = ctx->at<double>(ctx->L.staging);
    lbm::UtilArgs u;
    u.op = lbm::UTIL_WINDOW;
    u.runs = ctx->at<lbm::RunDev>(ctx->L.runs);
    u.run = run;
    u.nodes = (int64_t)w * h;
    u.f = ctx->fbuf(ctx->cur);
    u.psi = nullptr;
    u.buf = st;
    u.ux = u.uy = nullptr;
    u.parity = ctx->parity();
    // wrap the origin into the grid on periodic axes (psi_coord wraps once)
    u.wx0 = g.bc_x == LBM_BC_PERIODIC ? ((x0 % g.nx) + g.nx) % g.nx : x0;
    u.wy0 = g.bc_y == LBM_BC_PERIODIC ? ((y0 % g.ny) + g.ny) % g.ny : y0;
    u.ww = w;
    u.wh = h;
    u.stream = ctx->stream;
    if (ctx->precision == LBM_FP32_BF16STORE) {
        u.r0 = ctx->at<float>(ctx->L.r0);
        u.r1 = ctx->at<float>(ctx->L.r1);
    }
    LBM_HIP(lbm::launch_util(kernel_precision(ctx->precision), u));
    LBM_HIP(hipMemcpyAsync(f, st, sizeof(double) * 9 * (size_t)w * h, hipMemcpyDeviceToHost, ctx->stream));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_run_pressure(lbm_ctx *ctx, int32_t run, double *p)
{
    lbm::TraceRange trace_("lbm_run_pressure");
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!p) return fail(LBM_EINVAL, "null output");
    LBM_HIP(hipSetDevice(ctx->device));
    const int64_t N = run_nodes(ctx, run);
    double *st = ctx->at<double>(ctx->L.staging);
    if ((s = util(ctx, lbm::UTIL_PRESSURE, run, st)) != LBM_OK) return s;
    LBM_HIP(hipMemcpyAsync(p, st, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
    std::vector<int32_t> stt;
    if ((s = read_status(ctx, stt)) != LBM_OK) return s;
    return stt[run] ? fail(LBM_EDIVERGED, "run " + std::to_string(run) + " has diverged") : LBM_OK;
}

lbm_status lbm_run_get_populations(lbm_ctx *ctx, int32_t run, double *f)
{
    lbm::TraceRange trace_("lbm_run_get_populations");
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!f) return fail(LBM_EINVAL, "null output");
    LBM_HIP(hipSetDevice(ctx->device));
    const int64_t N = run_nodes(ctx, run);
    double *st = ctx->at<double>(ctx->L.staging);
    if ((s = util(ctx, lbm::UTIL_GET, run, st)) != LBM_OK) return s;
    LBM_HIP(hipMemcpyAsync(f, st, sizeof(double) * 9 * N, hipMemcpyDeviceToHost, ctx->stream));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx *ctx, double *f) { return lbm_run_get_populations(ctx, 0, f); }

lbm_status lbm_run_set_populations(lbm_ctx *ctx, int32_t run, const double *f)
{
    lbm::TraceRange trace_("lbm_run_set_populations");
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!f) return fail(LBM_EINVAL, "null input");
    const int64_t N = run_nodes(ctx, run);
    for (int64_t i = 0; i < 9 * N; ++i)
        if (!is_finite(f[i])) return fail(LBM_EINVAL, "populations must be finite");
    LBM_HIP(hipSetDevice(ctx->device));
    double *st = ctx->at<double>(ctx->L.staging);
    LBM_HIP(hipMemcpyAsync(st, f, sizeof(double) * 9 * N, hipMemcpyHostToDevice, ctx->stream));
    if ((s = util(ctx, lbm::UTIL_PUT, run, st)) != LBM_OK) return s;
    LBM_HIP(hipMemsetAsync(ctx->ws + ctx->L.status + sizeof(int32_t) * run, 0, sizeof(int32_t), ctx->stream));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx *ctx, const double *f) { return lbm_run_set_populations(ctx, 0, f); }

lbm_status lbm_run_set_multirange(lbm_ctx *ctx, int32_t run, double G1, double G2)
{
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!is_finite(G1) || !is_finite(G2) || G1 == 0.0) return fail(LBM_EINVAL, "G1 must be finite and non-zero");
    if (G2 != 0.0 && ctx->desc[run].kappa != 0.0)
        return fail(LBM_EINVAL, "the multi-range force needs kappa = 0 (Eq. 19 is defined for Eq. 7 only)");
    if (ctx->desc[run].eos.kind != LBM_EOS_SC_EXP && !(G1 + 2.0 * G2 < 0.0))
        return fail(LBM_EINVAL, "the sqrt psi forms need G1 + 2 G2 < 0");
    LBM_HIP(hipSetDevice(ctx->device));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    ctx->rdev[run].pd.G = G1;
    ctx->rdev[run].pd.G2 = G2;
    ctx->rdev[run].pd.G_eos = G1 + 2.0 * G2;
    int halo = 1;
    for (int i = 0; i < ctx->nruns; ++i)
        if (ctx->rdev[i].pd.G2 != 0.0) halo = 2;
    if (halo != ctx->halo) drop_graph(ctx); // the captured launches carry the tile halo
    ctx->halo = halo;
    if ((s = upload_run(ctx, run)) != LBM_OK) return s;
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_run_set_viscosity_step(lbm_ctx *ctx, int32_t run, double rho_threshold, double s_nu_low)
{
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!is_finite(rho_threshold) || rho_threshold < 0.0) return fail(LBM_EINVAL, "threshold must be finite and >= 0");
    if (rho_threshold > 0.0 && !(s_nu_low > 0.0 && s_nu_low < 2.0))
        return fail(LBM_EINVAL, "the low-density stress rate must lie in (0, 2)");
    LBM_HIP(hipSetDevice(ctx->device));
    ctx->rdev[run].pd.rho_nu = rho_threshold;
    ctx->rdev[run].pd.s_nu_low = rho_threshold > 0.0 ? s_nu_low : 0.0;
    // ordered after the work already on the stream; kernels read the table at launch
    if ((s = upload_run(ctx, run)) != LBM_OK) return s;
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_run_set_reference_density(lbm_ctx *ctx, int32_t run, double rho_ref)
{
    lbm_status s = check_run(ctx, run);
    if (s != LBM_OK) return s;
    if (!is_finite(rho_ref) || rho_ref < 0.0) return fail(LBM_EINVAL, "reference density must be finite and >= 0");
    if (ctx->precision == LBM_FP64) return fail(LBM_ESTATE, "FP64 storage keeps the populations themselves");
    if (ctx->precision == LBM_FP32_BF16STORE)
        return fail(LBM_ESTATE, "bf16 storage takes each population's base from the density of its writer");
    LBM_HIP(hipSetDevice(ctx->device));
    // decode with the old base into the staging area, re-encode with the new one
    double *st = ctx->at<double>(ctx->L.staging);
    if ((s = util(ctx, lbm::UTIL_GET, run, st)) != LBM_OK) return s;
    ctx->rdev[run].pd.rho_ref = rho_ref;
    ctx->ref_set[run] = 1;
    if ((s = upload_run(ctx, run)) != LBM_OK) return s;
    if ((s = util(ctx, lbm::UTIL_PUT, run, st)) != LBM_OK) return s;
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_batch_diagnostics(lbm_ctx *ctx, const lbm_region *regions, lbm_diag *out)
{
    lbm::TraceRange trace_("lbm_batch_diagnostics");
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (!regions || !out) return fail(LBM_EINVAL, "null argument");
    LBM_HIP(hipSetDevice(ctx->device));
    const int nr = ctx->nruns;
    std::vector<double> reg(4 * nr);
    for (int i = 0; i < nr; ++i) {
        if (!is_finite(regions[i].cx) || !is_finite(regions[i].cy) || !is_finite(regions[i].r_in) ||
            !is_finite(regions[i].r_out))
            return fail(LBM_EINVAL, "diagnostic regions must be finite");
        reg[4 * i] = regions[i].cx;
        reg[4 * i + 1] = regions[i].cy;
        reg[4 * i + 2] = regions[i].r_in;
        reg[4 * i + 3] = regions[i].r_out;
    }
    LBM_HIP(hipMemcpyAsync(ctx->ws + ctx->L.regions, reg.data(), sizeof(double) * 4 * nr, hipMemcpyHostToDevice,
                           ctx->stream));
    if ((s = refresh_psi(ctx)) != LBM_OK) return s;
    LBM_HIP(lbm::launch_diag(kernel_precision(ctx->precision), ctx->step_args(), ctx->at<double>(ctx->L.regions),
                             ctx->at<double>(ctx->L.partial), ctx->at<double>(ctx->L.dout), nr, ctx->parity()));
    std::vector<double> res(8 * nr);
    LBM_HIP(hipMemcpyAsync(res.data(), ctx->ws + ctx->L.dout, sizeof(double) * 8 * nr, hipMemcpyDeviceToHost,
                           ctx->stream));
    std::vector<int32_t> st;
    if ((s = read_status(ctx, st)) != LBM_OK) return s;
    bool any = false;
    for (int i = 0; i < nr; ++i) {
        const double *v = &res[8 * i];
        lbm_diag &d = out[i];
        const double N = (double)run_nodes(ctx, i);
        d.mass = v[0];
        d.rho_in = v[2] > 0 ? v[1] / v[2] : NAN;
        d.rho_out = v[4] > 0 ? v[3] / v[4] : NAN;
        d.p_in = v[2] > 0 ? v[5] / v[2] : NAN;
        d.p_out = v[4] > 0 ? v[6] / v[4] : NAN;
        d.dp = d.p_in - d.p_out;
        d.r_eq = std::sqrt((d.mass - d.rho_out * N) / (M_PI * (d.rho_in - d.rho_out)));
        d.max_speed = v[7];
        d.status = st[i];
        d.reserved = 0;
        any |= st[i] != 0;
    }
    return any ? fail(LBM_EDIVERGED, "at least one run has diverged") : LBM_OK;
}

lbm_status lbm_diagnostics(lbm_ctx *ctx, double cx, double cy, double r_in, double r_out, lbm_diag *out)
{
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (ctx->nruns != 1) return fail(LBM_ESTATE, "lbm_diagnostics needs a one-run context");
    lbm_region r{cx, cy, r_in, r_out};
    return lbm_batch_diagnostics(ctx, &r, out);
}

lbm_status lbm_run_status(lbm_ctx *ctx, int32_t *status)
{
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (!status) return fail(LBM_EINVAL, "null output");
    LBM_HIP(hipSetDevice(ctx->device));
    std::vector<int32_t> st;
    if ((s = read_status(ctx, st)) != LBM_OK) return s;
    bool any = false;
    for (int i = 0; i < ctx->nruns; ++i) {
        status[i] = st[i];
        any |= st[i] != 0;
    }
    return any ? fail(LBM_EDIVERGED, "at least one run has diverged") : LBM_OK;
}

// Checkpoint layout: 48-byte header {magic, precision, nruns, 0, steps,
// population bytes, 16 reserved bytes}, the per-run base densities, the raw
// population storage of the current state, then (bf16 storage) the writer
// densities of the current state and the last rounding seed, so that a
// restart continues bit for bit.  The state does not depend on the schedule
// (either buffer of the fused one holds it in the same layout).
static const uint32_t kMagic = 0x344d424cu; // "LBM4"

static uint64_t state_r_bytes(const lbm_ctx *c)
{
    return c->precision == LBM_FP32_BF16STORE ? sizeof(float) * (uint64_t)c->L.total_nodes + 8 : 0;
}

static uint64_t state_pop_bytes(const lbm_ctx *c) { return pop_bytes(c->precision) * (uint64_t)c->L.pop_elems; }

size_t lbm_state_bytes(const lbm_ctx *ctx)
{
    if (!ctx) return 0;
    return 48 + sizeof(double) * ctx->nruns + state_pop_bytes(ctx) + state_r_bytes(ctx);
}

lbm_status lbm_save_state(lbm_ctx *ctx, void *host_buf, size_t bytes)
{
    lbm::TraceRange trace_("lbm_save_state");
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (!host_buf || bytes < lbm_state_bytes(ctx)) return fail(LBM_EINVAL, "buffer smaller than lbm_state_bytes()");
    LBM_HIP(hipSetDevice(ctx->device));
    unsigned char *p = static_cast<unsigned char *>(host_buf);
    const uint64_t pb = state_pop_bytes(ctx);
    const uint32_t h[4] = {kMagic, (uint32_t)ctx->precision, (uint32_t)ctx->nruns, 0u};
    std::memset(p, 0, 48);
    std::memcpy(p, h, 16);
    std::memcpy(p + 16, &ctx->steps, 8);
    std::memcpy(p + 24, &pb, 8);
    unsigned char *q = p + 48;
    for (int i = 0; i < ctx->nruns; ++i, q += 8) std::memcpy(q, &ctx->rdev[i].pd.rho_ref, 8);
    LBM_HIP(hipMemcpyAsync(q, ctx->fbuf(ctx->cur), pb, hipMemcpyDeviceToHost, ctx->stream));
    if (state_r_bytes(ctx)) {
        // the current state decodes with R[parity ^ 1]; the last seed sits in slot parity ^ 1
        const int last = ctx->parity() ^ 1;
        const size_t rb = sizeof(float) * (size_t)ctx->L.total_nodes;
        LBM_HIP(hipMemcpyAsync(q + pb, ctx->ws + (last ? ctx->L.r1 : ctx->L.r0), rb, hipMemcpyDeviceToHost,
                               ctx->stream));
        LBM_HIP(hipMemcpyAsync(q + pb + rb, ctx->ws + ctx->L.seed + sizeof(uint32_t) * last, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, ctx->stream));
    }
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx *ctx, const void *host_buf, size_t bytes)
{
    lbm::TraceRange trace_("lbm_load_state");
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (!host_buf || bytes < 48) return fail(LBM_EINVAL, "checkpoint too short");
    const unsigned char *p = static_cast<const unsigned char *>(host_buf);
    uint32_t h[4];
    uint64_t pb;
    int64_t steps;
    std::memcpy(h, p, 16);
    std::memcpy(&steps, p + 16, 8);
    std::memcpy(&pb, p + 24, 8);
    if (h[0] != kMagic || h[1] != (uint32_t)ctx->precision || h[2] != (uint32_t)ctx->nruns ||
        pb != state_pop_bytes(ctx) || steps < 0)
        return fail(LBM_ESTATE, "checkpoint does not match this context");
    const uint64_t rbytes = state_r_bytes(ctx);
    if (bytes < 48 + 8 * (uint64_t)ctx->nruns + pb + rbytes) return fail(LBM_EINVAL, "checkpoint truncated");
    LBM_HIP(hipSetDevice(ctx->device));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    ctx->steps = steps;
    const unsigned char *q = p + 48;
    for (int i = 0; i < ctx->nruns; ++i, q += 8) std::memcpy(&ctx->rdev[i].pd.rho_ref, q, 8);
    for (int i = 0; i < ctx->nruns; ++i) lbm::finish_rundev(ctx->rdev[i]);
    LBM_HIP(hipMemcpyAsync(ctx->ws + ctx->L.runs, ctx->rdev.data(), sizeof(lbm::RunDev) * ctx->nruns,
                           hipMemcpyHostToDevice, ctx->stream));
    LBM_HIP(hipMemcpyAsync(ctx->fbuf(ctx->cur), q, pb, hipMemcpyHostToDevice, ctx->stream));
    if (rbytes) {
        // the writer densities decode the current state; the last seed sits in slot parity ^ 1
        const int last = ctx->parity() ^ 1;
        const size_t rb = sizeof(float) * (size_t)ctx->L.total_nodes;
        LBM_HIP(hipMemcpyAsync(ctx->ws + (last ? ctx->L.r1 : ctx->L.r0), q + pb, rb, hipMemcpyHostToDevice,
                               ctx->stream));
        LBM_HIP(hipMemcpyAsync(ctx->ws + ctx->L.seed + sizeof(uint32_t) * last, q + pb + rb, sizeof(uint32_t),
                               hipMemcpyHostToDevice, ctx->stream));
    }
    LBM_HIP(hipMemsetAsync(ctx->ws + ctx->L.status, 0, sizeof(int32_t) * ctx->nruns, ctx->stream));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

lbm_status lbm_set_graph_steps(lbm_ctx *ctx, int32_t k)
{
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (k < 0 || k > 4096) return fail(LBM_EINVAL, "graph steps must lie in [0, 4096]");
    LBM_HIP(hipSetDevice(ctx->device));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph(ctx);
    ctx->graph_k = k;
    ctx->graph_failed = false;
    return LBM_OK;
}

lbm_status lbm_set_tile(lbm_ctx *ctx, int32_t tx, int32_t ty)
{
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (!tile_allowed(tx, ty)) return fail(LBM_EINVAL, "tile shape not supported");
    LBM_HIP(hipSetDevice(ctx->device));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph(ctx);
    ctx->tx = tx;
    ctx->ty = ty;
    build_tiles(ctx);
    return upload_tables(ctx);
}

lbm_status lbm_time_kernels(lbm_ctx *ctx, int64_t n, double *psi_ms, double *collide_ms)
{
    lbm::TraceRange trace_("lbm_time_kernels");
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (n < 1 || !psi_ms || !collide_ms) return fail(LBM_EINVAL, "need n >= 1 and two outputs");
    LBM_HIP(hipSetDevice(ctx->device));
    const int prec = kernel_precision(ctx->precision);
    // the start/stop events are attached to the dispatch itself, so each pair
    // brackets exactly one kernel's execution
    std::vector<hipEvent_t> ev(4 * n, nullptr);
    lbm_status rc = LBM_OK;
    int64_t made = 0;
    for (; made < 4 * n; ++made) {
        hipError_t e = hipEventCreate(&ev[made]);
        if (e != hipSuccess) {
            rc = fail(LBM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
            break;
        }
    }
    double tp = 0.0, tc = 0.0;
    if (rc == LBM_OK) {
        hipError_t e = hipSuccess;
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) {
            const int par = ctx->parity();
            lbm::StepArgs a = ctx->step_args();
            if (ctx->fused) {
                // one kernel per step: the psi pair brackets an empty interval
                e = hipEventRecord(ev[4 * i], ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(ev[4 * i + 1], ctx->stream);
                a.ev_start = ev[4 * i + 2];
                a.ev_stop = ev[4 * i + 3];
                if (e == hipSuccess) e = lbm::launch_fused(prec, a, par);
                if (e == hipSuccess) ctx->cur ^= 1;
            } else {
                a.ev_start = ev[4 * i];
                a.ev_stop = ev[4 * i + 1];
                e = lbm::launch_psi(prec, a, par);
                a.ev_start = ev[4 * i + 2];
                a.ev_stop = ev[4 * i + 3];
                if (e == hipSuccess) e = lbm::launch_collide(prec, a, par);
            }
            if (e == hipSuccess) ++ctx->steps;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) {
            float a1 = 0.f, a2 = 0.f;
            e = hipEventElapsedTime(&a1, ev[4 * i], ev[4 * i + 1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&a2, ev[4 * i + 2], ev[4 * i + 3]);
            tp += a1;
            tc += a2;
        }
        if (e != hipSuccess) rc = fail(LBM_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
    }
    for (int64_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (rc == LBM_OK) {
        *psi_ms = ctx->fused ? 0.0 : tp / n;
        *collide_ms = tc / n;
    }
    return rc;
}

lbm_status lbm_set_fused(lbm_ctx *ctx, int32_t rows)
{
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (rows != 0 && rows != 1 && rows != 2 && rows != 4) return fail(LBM_EINVAL, "fused must be 0, 1, 2 or 4");
    LBM_HIP(hipSetDevice(ctx->device));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph(ctx);
    ctx->fused = rows;
    build_tiles(ctx);
    return upload_tables(ctx);
}

lbm_status lbm_autotune(lbm_ctx *ctx, int32_t steps, int32_t *tx, int32_t *ty, int32_t *fused)
{
    lbm::TraceRange trace_("lbm_autotune");
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    if (steps < 2) return fail(LBM_EINVAL, "autotune needs at least 2 steps per candidate");
    LBM_HIP(hipSetDevice(ctx->device));
    struct Cand {
        int tx, ty, fused;
    };
    const Cand cands[] = {{64, 4, 0}, {128, 2, 0}, {32, 8, 0}, {256, 1, 0}, {64, 2, 0}, {32, 4, 0}, {64, 4, 1},
                          {64, 4, 2}, {64, 4, 4}, {128, 2, 2}, {128, 2, 4}, {256, 1, 4}, {32, 8, 2}, {64, 2, 4},
                          {256, 2, 4}, {128, 4, 2}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LBM_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LBM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(he));
    }
    float best = 0.f;
    Cand pick = {ctx->tx, ctx->ty, ctx->fused};
    lbm_status rc = LBM_OK;
    const int64_t n = steps + (steps & 1);
    for (const Cand &c : cands) {
        if ((rc = lbm_set_tile(ctx, c.tx, c.ty)) != LBM_OK) break;
        if ((rc = lbm_set_fused(ctx, c.fused)) != LBM_OK) break;
        // one untimed replay builds the graph
        if ((rc = lbm_step(ctx, 2 * (int64_t)std::max(ctx->graph_k, 1))) != LBM_OK) break;
        he = hipEventRecord(e0, ctx->stream);
        if (he == hipSuccess && (rc = lbm_step(ctx, n)) != LBM_OK) break;
        if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            rc = fail(LBM_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(he));
            break;
        }
        if (best == 0.f || ms < best) {
            best = ms;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) return rc;
    if ((rc = lbm_set_tile(ctx, pick.tx, pick.ty)) != LBM_OK) return rc;
    if ((rc = lbm_set_fused(ctx, pick.fused)) != LBM_OK) return rc;
    if (tx) *tx = pick.tx;
    if (ty) *ty = pick.ty;
    if (fused) *fused = pick.fused;
    return LBM_OK;
}

lbm_status lbm_set_xcd_order(lbm_ctx *ctx, int32_t on)
{
    lbm_status s = check_ctx(ctx);
    if (s != LBM_OK) return s;
    LBM_HIP(hipSetDevice(ctx->device));
    LBM_HIP(hipStreamSynchronize(ctx->stream));
    drop_graph(ctx);
    ctx->xcd = on ? 1 : 0;
    return LBM_OK;
}

lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, int32_t reps, void *stream, double *ms)
{
    if (!dst || !src || !ms || reps < 1 || bytes == 0 || (bytes & 15) ||
        (reinterpret_cast<uintptr_t>(dst) & 15) || (reinterpret_cast<uintptr_t>(src) & 15))
        return fail(LBM_EINVAL, "copy needs 16-byte aligned pointers, a 16-byte multiple and reps >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    bool own = false;
    if (!st) {
        LBM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        own = true;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = lbm::launch_copy(dst, src, bytes, st); // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = lbm::launch_copy(dst, src, bytes, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (own) (void)hipStreamDestroy(st);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("stream copy: ") + hipGetErrorString(e));
    *ms = (double)t / reps;
    return LBM_OK;
}

} // extern "C"

// ------------------------------------------------ allocation-free step
// Scratch of lbm_step_noalloc: psi of up to kNoAllocNodes FP64 nodes, the run
// record, up to kNoAllocTiles work-list tiles and a status flag, in one
// file-scope device array (33 MiB), one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel: it is a
// host-side stand-in, not a device address; kernels get the address that
// hipGetSymbolAddress returned for the current device.
namespace {

constexpr int64_t kNoAllocNodes = int64_t(1) << 22;
constexpr int64_t kNoAllocTiles = int64_t(1) << 16;
constexpr int kNoAllocTx = 64, kNoAllocTy = 4;
constexpr size_t kScratchPsi = 0;
constexpr size_t kScratchRun = kScratchPsi + sizeof(double) * kNoAllocNodes;
constexpr size_t kScratchTiles = kScratchRun + 512;
constexpr size_t kScratchStatus = kScratchTiles + sizeof(lbm::Tile) * kNoAllocTiles;
constexpr size_t kScratchBytes = kScratchStatus + 256;
static_assert(sizeof(lbm::RunDev) <= 512, "run record fits its scratch slot");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

} // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.
lbm_status scratch_of_current_device(unsigned char **out)
{
    int dev = 0;
    LBM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

} // namespace

extern "C" lbm_status lbm_step_noalloc(const lbm_grid *grid, const lbm_eos *eos, double G, const lbm_rates *rates,
                                       double kappa, double epsilon, double *f, int64_t t0, int64_t n,
                                       int32_t *status, void *stream)
{
    lbm::TraceRange trace_("lbm_step_noalloc");
    if (!grid || !eos || !rates) return fail(LBM_EINVAL, "null argument");
    lbm_run_desc d;
    d.grid = *grid;
    d.eos = *eos;
    d.G = G;
    d.rates = *rates;
    d.kappa = kappa;
    d.epsilon = epsilon;
    lbm_status s = validate_run(&d);
    if (s != LBM_OK) return s;
    if (!f) return fail(LBM_EINVAL, "null population array");
    if (t0 < 0 || n < 0) return fail(LBM_EINVAL, "step counts must be >= 0");
    const int64_t nodes = (int64_t)grid->nx * grid->ny;
    if (nodes > kNoAllocNodes)
        return fail(LBM_EINVAL, "grid of " + std::to_string(nodes) + " nodes exceeds the allocation-free maximum of " +
                                    std::to_string(kNoAllocNodes));
    const int ntx = (grid->nx + kNoAllocTx - 1) / kNoAllocTx, nty = (grid->ny + kNoAllocTy - 1) / kNoAllocTy;
    const int64_t ntiles = (int64_t)ntx * nty;
    if (ntiles > kNoAllocTiles)
        return fail(LBM_EINVAL, "grid needs " + std::to_string(ntiles) + " tiles of 64 x 4, more than the " +
                                    std::to_string(kNoAllocTiles) + " of the allocation-free scratch");
    if (n == 0) return LBM_OK;
    unsigned char *base = nullptr;
    if ((s = scratch_of_current_device(&base)) != LBM_OK) return s;
    // the caller's populations are a dense [9][ny][nx] array
    lbm::RunDev r = make_rundev(d);
    r.pitch = grid->nx;
    r.dstride = nodes;
    r.f_off = 0;
    r.n_off = 0;
    r.tile_begin = 0;
    r.tile_count = (int32_t)ntiles;
    lbm::finish_rundev(r);
    hipStream_t st = static_cast<hipStream_t>(stream);
    lbm::RunDev *runs = reinterpret_cast<lbm::RunDev *>(base + kScratchRun);
    lbm::Tile *tiles = reinterpret_cast<lbm::Tile *>(base + kScratchTiles);
    int32_t *stat = status ? status : reinterpret_cast<int32_t *>(base + kScratchStatus);
    LBM_HIP(lbm::launch_table_setup(r, runs, tiles, ntx, (int)ntiles, kNoAllocTx, kNoAllocTy, stat, st));
    lbm::StepArgs a;
    a.runs = runs;
    a.tiles = tiles;
    a.ntiles = (int)ntiles;
    a.tx = kNoAllocTx;
    a.ty = kNoAllocTy;
    a.f = f;
    a.psi = base + kScratchPsi;
    a.status = stat;
    a.stream = st;
    a.xcd = 1;
    a.fused = 0; // in place: psi pass, then collide and stream
    a.halo = 1;
    for (int64_t i = 0; i < n; ++i) LBM_HIP(lbm::launch_step(lbm::PREC_FP64, a, (int)((t0 + i) & 1)));
    return LBM_OK;
}

void lbm::set_last_error(const std::string &msg) { g_error = msg; }
