// HIP kernels (gfx950) of the D2Q9 pseudopotential MRT lattice Boltzmann step
// with the surface-tension source term of Li & Luo (arXiv:1306.6445).
//
// One step = two launches over the tile work list of every run in a context:
//   psi_kernel      rho = sum_a f_a (Eq. 6) -> psi(rho) (Section II, Eq. 23)
//   collide_kernel  psi tile + halo in LDS -> F (Eq. 7), Q (Eq. 19) -> v (Eq. 6)
//                   -> m = M f, m_eq (Eq. 3), S (Eqs. 5, 8), C (Eq. 18)
//                   -> m* (Eq. 17) -> f* = M^-1 m* -> in-place AA store (Eq. 4)
// Both are HBM-bound streaming kernels: one thread per node, nine coalesced
// structure-of-arrays loads and stores, moment transforms as add chains.
#include <hip/hip_ext.h>

#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// ----------------------------------------------------------------- helpers

template <typename S, int PARITY>
struct LoadPops {
    using C = typename Store<S>::C;
    const S *fb;
    int x, y, nx;
    int64_t N;
    const Nbr *n;
    C ref;
    C *f;
    template <int A> __device__ __forceinline__ void operator()()
    {
        const int64_t i = PARITY == 0 ? even_slot<A>(x, y, nx, N) : odd_slot<A>(x, y, *n, nx, N);
        f[A] = Store<S>::template load<A>(fb, i, ref);
    }
};

template <typename S, int PARITY>
struct StorePops {
    using C = typename Store<S>::C;
    S *fb;
    int x, y, nx;
    int64_t N;
    const Nbr *n;
    C ref;
    const C *f;
    template <int A> __device__ __forceinline__ void operator()()
    {
        constexpr int B = opp_of(A);
        // even step: f*_A goes to slot opp(A) of this node;
        // odd step: f*_A goes where the odd-state rule keeps f_opp(A) of this node.
        const int64_t i = PARITY == 0 ? even_slot<B>(x, y, nx, N) : odd_slot<B>(x, y, *n, nx, N);
        Store<S>::template store<A>(fb, i, f[A], ref);
    }
};

template <typename S, int PARITY>
__device__ __forceinline__ void load_node(const S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                          typename Store<S>::C ref, typename Store<S>::C *f)
{
    LoadPops<S, PARITY> op{fb, x, y, nx, N, &n, ref, f};
    for9(op);
}

template <typename S, int PARITY>
__device__ __forceinline__ void store_node(S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                           typename Store<S>::C ref, const typename Store<S>::C *f)
{
    StorePops<S, PARITY> op{fb, x, y, nx, N, &n, ref, f};
    for9(op);
}

// Runtime-parity variants for the (non-hot) utility kernels.
template <typename S>
__device__ __forceinline__ void load_node_rt(const S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                             typename Store<S>::C ref, typename Store<S>::C *f, int parity)
{
    if (parity == 0)
        load_node<S, 0>(fb, x, y, nx, N, n, ref, f);
    else
        load_node<S, 1>(fb, x, y, nx, N, n, ref, f);
}

// Location of f_a(x) in the current state (put/get kernels).
template <typename S, int PARITY>
struct PutPops {
    using C = typename Store<S>::C;
    S *fb;
    int x, y, nx;
    int64_t N;
    const Nbr *n;
    C ref;
    const C *f;
    template <int A> __device__ __forceinline__ void operator()()
    {
        const int64_t i = PARITY == 0 ? even_slot<A>(x, y, nx, N) : odd_slot<A>(x, y, *n, nx, N);
        Store<S>::template store<A>(fb, i, f[A], ref);
    }
};

template <typename S>
__device__ __forceinline__ void put_node_rt(S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                            typename Store<S>::C ref, const typename Store<S>::C *f, int parity)
{
    if (parity == 0) {
        PutPops<S, 0> op{fb, x, y, nx, N, &n, ref, f};
        for9(op);
    } else {
        PutPops<S, 1> op{fb, x, y, nx, N, &n, ref, f};
        for9(op);
    }
}

// f = M^-1 m for the orthogonal D2Q9 basis (rho, e, zeta, jx, qx, jy, qy, pxx, pxy):
// M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
template <typename C>
__device__ __forceinline__ void moments_to_pops(const C *m, C *f)
{
    const C a = m[0] * C(1.0 / 9.0), b = m[1] * C(1.0 / 36.0), c = m[2] * C(1.0 / 36.0);
    const C d = m[3] * C(1.0 / 6.0), e = m[4] * C(1.0 / 12.0), g = m[5] * C(1.0 / 6.0);
    const C h = m[6] * C(1.0 / 12.0), i = m[7] * C(0.25), j = m[8] * C(0.25);
    const C ax = a - b - C(2) * c; // common part of the axis populations
    const C dg = a + C(2) * b + c; // common part of the diagonal populations
    f[0] = a - C(4) * b + C(4) * c;
    f[1] = ax + d - C(2) * e + i;
    f[2] = ax + g - C(2) * h - i;
    f[3] = ax - d + C(2) * e + i;
    f[4] = ax - g + C(2) * h - i;
    const C de = d + e, gh = g + h;
    f[5] = dg + de + gh + j;
    f[6] = dg - de + gh - j;
    f[7] = dg - de - gh + j;
    f[8] = dg + de - gh - j;
}

template <typename C>
__device__ __forceinline__ void equilibrium_moments(C rho, C vx, C vy, C *m)
{
    const C v2 = vx * vx + vy * vy;
    m[0] = rho;
    m[1] = rho * (C(-2) + C(3) * v2);
    m[2] = rho * (C(1) - C(3) * v2);
    m[3] = rho * vx;
    m[4] = -rho * vx;
    m[5] = rho * vy;
    m[6] = -rho * vy;
    m[7] = rho * (vx * vx - vy * vy);
    m[8] = rho * vx * vy;
}

// ----------------------------------------------------------- psi kernel

template <typename S, int PARITY>
__global__ void __launch_bounds__(256) psi_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                           const S *__restrict__ f, typename Store<S>::C *__restrict__ psi,
                           int32_t *__restrict__ status, int xcd)
{
    using C = typename Store<S>::C;
    const Tile t = tiles[work_index(xcd)];
    const RunDev &r = runs[t.run];
    const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y;
    const int nx = r.nx, ny = r.ny;
    if (x >= nx || y >= ny) return;
    const int64_t N = (int64_t)nx * ny;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    C fv[9];
    load_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, C(r.rho_ref), fv);
    // Eq. (6): rho = sum_a f_a
    const C rho = ((fv[0] + (fv[1] + fv[3])) + (fv[2] + fv[4])) + ((fv[5] + fv[7]) + (fv[6] + fv[8]));
    C ps;
    if (!eval_psi<C>(r, rho, ps)) {
        status[t.run] = 1;
        ps = C(NAN);
    }
    psi[r.n_off + (int64_t)y * nx + x] = ps;
}

// ------------------------------------------------------- collide kernel

template <typename S, int PARITY>
__global__ void __launch_bounds__(256) collide_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                               S *__restrict__ f, const typename Store<S>::C *__restrict__ psi, int xcd)
{
    using C = typename Store<S>::C;
    extern __shared__ unsigned char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);

    const Tile t = tiles[work_index(xcd)];
    const RunDev &r = runs[t.run];
    const int nx = r.nx, ny = r.ny;
    const int TX = blockDim.x, TY = blockDim.y;
    const int LX = TX + 2, LY = TY + 2;
    const C *pb = psi + r.n_off;

    // psi of the tile plus a one-node halo, wrapped or clamped per boundary
    for (int i = threadIdx.y * TX + threadIdx.x; i < LX * LY; i += TX * TY) {
        const int ly = i / LX, lx = i - ly * LX;
        const int gx = psi_coord(t.x0 - 1 + lx, nx, r.bc_x);
        const int gy = psi_coord(t.y0 - 1 + ly, ny, r.bc_y);
        lds[i] = pb[(int64_t)gy * nx + gx];
    }
    __syncthreads();

    const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int64_t N = (int64_t)nx * ny;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    const C ref = C(r.rho_ref);
    C fv[9];
    load_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, ref, fv);

    // psi at x + e_a from LDS
    const C *lc = lds + (threadIdx.y + 1) * LX + (threadIdx.x + 1);
    const C p0 = lc[0];
    const C p1 = lc[1], p3 = lc[-1], p2 = lc[LX], p4 = lc[-LX];
    const C p5 = lc[LX + 1], p6 = lc[LX - 1], p7 = lc[-LX - 1], p8 = lc[-LX + 1];

    const C G = C(r.G);
    // Eq. (7): F = -G psi(x) sum_a w_a psi(x + e_a) e_a, w = 1/3 (axis), 1/12 (diagonal)
    const C sx = C(1.0 / 3.0) * (p1 - p3) + C(1.0 / 12.0) * ((p5 - p7) + (p8 - p6));
    const C sy = C(1.0 / 3.0) * (p2 - p4) + C(1.0 / 12.0) * ((p5 - p7) + (p6 - p8));
    const C Fx = -G * p0 * sx, Fy = -G * p0 * sy;
    // Eq. (19): Q = kappa G/2 psi(x) sum_a w_a [psi(x + e_a) - psi(x)] e_a e_a
    const C dsum = (p5 + p6) + (p7 + p8) - C(4) * p0;
    const C kq = C(r.kappa) * G * C(0.5) * p0;
    const C Qxx = kq * (C(1.0 / 3.0) * (p1 + p3 - C(2) * p0) + C(1.0 / 12.0) * dsum);
    const C Qyy = kq * (C(1.0 / 3.0) * (p2 + p4 - C(2) * p0) + C(1.0 / 12.0) * dsum);
    const C Qxy = kq * (C(1.0 / 12.0) * ((p5 + p7) - (p6 + p8)));

    // Eq. (6): density and velocity (with F/2)
    const C sA = fv[1] + fv[3], sB = fv[2] + fv[4], sD = (fv[5] + fv[7]) + (fv[6] + fv[8]);
    const C rho = (fv[0] + sA) + sB + sD;
    const C d13 = fv[1] - fv[3], d24 = fv[2] - fv[4];
    const C d57 = fv[5] - fv[7], d86 = fv[8] - fv[6];
    const C jx = d13 + (d57 + d86);
    const C jy = d24 + (d57 - d86);
    const C irho = C(1) / rho;
    const C vx = (jx + C(0.5) * Fx) * irho, vy = (jy + C(0.5) * Fy) * irho;

    // m = M f (non-conserved moments)
    const C sAB = sA + sB;
    const C m1 = C(-4) * fv[0] - sAB + C(2) * sD;
    const C m2 = C(4) * fv[0] - C(2) * sAB + sD;
    const C qdx = d57 + d86, qdy = d57 - d86;
    const C m4 = C(-2) * d13 + qdx;
    const C m6 = C(-2) * d24 + qdy;
    const C m7 = sA - sB;
    const C m8 = (fv[5] + fv[7]) - (fv[6] + fv[8]);

    // Eq. (3) equilibria
    const C vxx = vx * vx, vyy = vy * vy, v2 = vxx + vyy;
    const C e1 = rho * (C(-2) + C(3) * v2), e2 = rho * (C(1) - C(3) * v2);
    const C e7 = rho * (vxx - vyy), e8 = rho * vx * vy;

    // Eqs. (5), (8): S1 = 6 v.F + 12 sigma |F|^2 / (psi^2 (tau_e - 1/2));
    // |F|^2 / psi^2 = G^2 (sx^2 + sy^2) exactly.
    const C S1 = C(6) * (vx * Fx + vy * Fy) + C(r.sig_coef) * G * G * (sx * sx + sy * sy);
    const C S7 = C(2) * (vx * Fx - vy * Fy);
    const C S8 = vx * Fy + vy * Fx;
    // Eq. (18)
    const C trQ = Qxx + Qyy;
    const C se = C(r.s_e), sz = C(r.s_zeta), sq = C(r.s_q), sv = C(r.s_nu);
    const C C1 = C(1.5) * se * trQ, C2 = C(-1.5) * sz * trQ;
    const C C7 = -sv * (Qxx - Qyy), C8 = -sv * Qxy;

    // Eq. (17).  Conserved moments: m*_rho = rho, and with the Eq. (6) velocity
    // j* = j - s_j (j - rho v) + (1 - s_j/2) F = j + F for any s_j.
    C ms[9];
    ms[0] = rho;
    ms[1] = m1 - se * (m1 - e1) + (C(1) - C(0.5) * se) * S1 + C1;
    ms[2] = m2 - sz * (m2 - e2) - (C(1) - C(0.5) * sz) * S1 + C2;
    ms[3] = jx + Fx;
    ms[4] = m4 - sq * (m4 + rho * vx) - (C(1) - C(0.5) * sq) * Fx;
    ms[5] = jy + Fy;
    ms[6] = m6 - sq * (m6 + rho * vy) - (C(1) - C(0.5) * sq) * Fy;
    ms[7] = m7 - sv * (m7 - e7) + (C(1) - C(0.5) * sv) * S7 + C7;
    ms[8] = m8 - sv * (m8 - e8) + (C(1) - C(0.5) * sv) * S8 + C8;

    C fs[9];
    moments_to_pops<C>(ms, fs);
    store_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, ref, fs);
}

// ------------------------------------------------------- utility kernels
// These run once per call of the host API (initialisation, read-back,
// diagnostics); one thread per node of a single run.

__device__ __forceinline__ bool node_of(const RunDev &r, int64_t idx, int &x, int &y)
{
    if (idx >= (int64_t)r.nx * r.ny) return false;
    y = (int)(idx / r.nx);
    x = (int)(idx - (int64_t)y * r.nx);
    return true;
}

// Equilibrium initialisation f = M^-1 m_eq(rho, u) (Eq. 3) from FP64 fields.
template <typename S>
__global__ void init_kernel(const RunDev *__restrict__ runs, int run, S *__restrict__ f,
                            const double *__restrict__ rho, const double *__restrict__ ux,
                            const double *__restrict__ uy, int parity)
{
    using C = typename Store<S>::C;
    const RunDev &r = runs[run];
    int x, y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!node_of(r, idx, x, y)) return;
    const double vx = ux ? ux[idx] : 0.0, vy = uy ? uy[idx] : 0.0;
    double m[9], fd[9];
    equilibrium_moments<double>(rho[idx], vx, vy, m);
    moments_to_pops<double>(m, fd);
    C fc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fc[a] = (C)fd[a];
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    put_node_rt<S>(f + r.f_off, x, y, r.nx, (int64_t)r.nx * r.ny, n, C(r.rho_ref), fc, parity);
}

// Canonical FP64 populations [9][ny][nx] -> storage at the current parity.
template <typename S>
__global__ void put_kernel(const RunDev *__restrict__ runs, int run, S *__restrict__ f,
                           const double *__restrict__ src, int parity)
{
    using C = typename Store<S>::C;
    const RunDev &r = runs[run];
    int x, y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!node_of(r, idx, x, y)) return;
    const int64_t N = (int64_t)r.nx * r.ny;
    C fc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fc[a] = (C)src[a * N + idx];
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    put_node_rt<S>(f + r.f_off, x, y, r.nx, N, n, C(r.rho_ref), fc, parity);
}

// Storage at the current parity -> canonical FP64 populations [9][ny][nx].
template <typename S>
__global__ void get_kernel(const RunDev *__restrict__ runs, int run, const S *__restrict__ f,
                           double *__restrict__ dst, int parity)
{
    using C = typename Store<S>::C;
    const RunDev &r = runs[run];
    int x, y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!node_of(r, idx, x, y)) return;
    const int64_t N = (int64_t)r.nx * r.ny;
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, r.nx, N, n, C(r.rho_ref), fc, parity);
#pragma unroll
    for (int a = 0; a < 9; ++a) dst[a * N + idx] = (double)fc[a];
}

// Density and Eq. (6) velocity of one run in FP64, using psi of the current state.
template <typename S>
__device__ __forceinline__ void node_macro(const RunDev &r, const S *f, const typename Store<S>::C *psi,
                                           int x, int y, int parity, double &rho, double &vx, double &vy)
{
    using C = typename Store<S>::C;
    const int nx = r.nx, ny = r.ny;
    const int64_t N = (int64_t)nx * ny;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, nx, N, n, C(r.rho_ref), fc, parity);
    double fd[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fd[a] = (double)fc[a];
    rho = ((fd[0] + (fd[1] + fd[3])) + (fd[2] + fd[4])) + ((fd[5] + fd[7]) + (fd[6] + fd[8]));
    const double jx = (fd[1] - fd[3]) + ((fd[5] - fd[7]) + (fd[8] - fd[6]));
    const double jy = (fd[2] - fd[4]) + ((fd[5] - fd[7]) + (fd[6] - fd[8]));
    const C *pb = psi + r.n_off;
    auto P = [&](int dx, int dy) -> double {
        const int gx = psi_coord(x + dx, nx, r.bc_x), gy = psi_coord(y + dy, ny, r.bc_y);
        return (double)pb[(int64_t)gy * nx + gx];
    };
    const double p0 = P(0, 0);
    const double sx = (P(1, 0) - P(-1, 0)) / 3.0 + ((P(1, 1) - P(-1, -1)) + (P(1, -1) - P(-1, 1))) / 12.0;
    const double sy = (P(0, 1) - P(0, -1)) / 3.0 + ((P(1, 1) - P(-1, -1)) + (P(-1, 1) - P(1, -1))) / 12.0;
    const double Fx = -r.G * p0 * sx, Fy = -r.G * p0 * sy;
    vx = (jx + 0.5 * Fx) / rho;
    vy = (jy + 0.5 * Fy) / rho;
}

template <typename S>
__global__ void moments_kernel(const RunDev *__restrict__ runs, int run, const S *__restrict__ f,
                               const typename Store<S>::C *__restrict__ psi, double *__restrict__ out,
                               int parity)
{
    const RunDev &r = runs[run];
    int x, y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!node_of(r, idx, x, y)) return;
    double rho, vx, vy;
    node_macro<S>(r, f, psi, x, y, parity, rho, vx, vy);
    const int64_t N = (int64_t)r.nx * r.ny;
    out[idx] = rho;
    out[N + idx] = vx;
    out[2 * N + idx] = vy;
}

// Droplet diagnostics: per-tile FP64 partial sums, then a per-run reduction.
// Partial layout (8 doubles): mass, sum rho_in, n_in, sum rho_out, n_out,
// sum p_in, sum p_out, max speed.
constexpr int DIAG_THREADS = 256;

template <typename S>
__global__ void __launch_bounds__(DIAG_THREADS)
diag_partial_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, const S *__restrict__ f,
                    const typename Store<S>::C *__restrict__ psi, const double *__restrict__ regions,
                    double *__restrict__ partial, int parity, int xcd)
{
    __shared__ double red[8][DIAG_THREADS];
    const int wi = work_index(xcd);
    const Tile t = tiles[wi];
    const RunDev &r = runs[t.run];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y;
    if (x < r.nx && y < r.ny) {
        double rho, vx, vy;
        node_macro<S>(r, f, psi, x, y, parity, rho, vx, vy);
        const double cx = regions[4 * t.run], cy = regions[4 * t.run + 1];
        const double r_in = regions[4 * t.run + 2], r_out = regions[4 * t.run + 3];
        // minimum-image distance on periodic axes
        double dx = x - cx, dy = y - cy;
        if (r.bc_x == BC_PERIODIC) dx -= r.nx * rint(dx / r.nx);
        if (r.bc_y == BC_PERIODIC) dy -= r.ny * rint(dy / r.ny);
        const double dist = sqrt(dx * dx + dy * dy);
        const double p = eval_pressure(r, rho);
        v[0] = rho;
        if (dist <= r_in) {
            v[1] = rho;
            v[2] = 1.0;
            v[5] = p;
        }
        if (dist >= r_out) {
            v[3] = rho;
            v[4] = 1.0;
            v[6] = p;
        }
        const double sp = sqrt(vx * vx + vy * vy);
        v[7] = sp == sp ? sp : INFINITY;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[k][tid] = v[k];
    __syncthreads();
    const int nt = blockDim.x * blockDim.y;
    for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s && tid + s < nt) {
#pragma unroll
            for (int k = 0; k < 7; ++k) red[k][tid] += red[k][tid + s];
            red[7][tid] = fmax(red[7][tid], red[7][tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) partial[(int64_t)wi * 8 + k] = red[k][0];
    }
}

// One block per run: reduce that run's tile partials in a fixed order.
__global__ void __launch_bounds__(256)
diag_final_kernel(const RunDev *__restrict__ runs, const double *__restrict__ partial, double *__restrict__ out)
{
    __shared__ double red[8][256];
    const RunDev &r = runs[blockIdx.x];
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < r.tile_count; i += blockDim.x) {
        const double *p = partial + (int64_t)(r.tile_begin + i) * 8;
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] += p[k];
        v[7] = fmax(v[7], p[7]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 7; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
            red[7][threadIdx.x] = fmax(red[7][threadIdx.x], red[7][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) out[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// ------------------------------------------------------------ launchers

template <typename S>
hipError_t launch_psi_t(const StepArgs &a, int parity)
{
    using C = typename Store<S>::C;
    const dim3 block(a.tx, a.ty);
    S *f = static_cast<S *>(a.f);
    C *psi = static_cast<C *>(a.psi);
    if (parity == 0)
        hipExtLaunchKernelGGL(psi_kernel<S, 0>, dim3(a.ntiles), block, 0, a.stream, a.ev_start, a.ev_stop, 0,
                              a.runs, a.tiles, (const S *)f, psi, a.status, a.xcd);
    else
        hipExtLaunchKernelGGL(psi_kernel<S, 1>, dim3(a.ntiles), block, 0, a.stream, a.ev_start, a.ev_stop, 0,
                              a.runs, a.tiles, (const S *)f, psi, a.status, a.xcd);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_collide_t(const StepArgs &a, int parity)
{
    using C = typename Store<S>::C;
    const dim3 block(a.tx, a.ty);
    const uint32_t lds = sizeof(C) * (a.tx + 2) * (a.ty + 2);
    S *f = static_cast<S *>(a.f);
    const C *psi = static_cast<const C *>(a.psi);
    if (parity == 0)
        hipExtLaunchKernelGGL(collide_kernel<S, 0>, dim3(a.ntiles), block, lds, a.stream, a.ev_start, a.ev_stop,
                              0, a.runs, a.tiles, f, psi, a.xcd);
    else
        hipExtLaunchKernelGGL(collide_kernel<S, 1>, dim3(a.ntiles), block, lds, a.stream, a.ev_start, a.ev_stop,
                              0, a.runs, a.tiles, f, psi, a.xcd);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_step_t(const StepArgs &a, int parity)
{
    StepArgs b = a;
    b.ev_start = b.ev_stop = nullptr;
    hipError_t e = launch_psi_t<S>(b, parity);
    return e == hipSuccess ? launch_collide_t<S>(b, parity) : e;
}

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename S>
hipError_t launch_util_t(const UtilArgs &u)
{
    using C = typename Store<S>::C;
    const int bs = 256;
    const unsigned nb = blocks_for(u.nodes, bs);
    S *f = static_cast<S *>(u.f);
    switch (u.op) {
    case UTIL_INIT:
        init_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, u.buf, u.ux, u.uy, u.parity);
        break;
    case UTIL_PUT:
        put_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, u.buf, u.parity);
        break;
    case UTIL_GET:
        get_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, u.buf, u.parity);
        break;
    case UTIL_MOMENTS:
        moments_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, static_cast<const C *>(u.psi), u.buf,
                                                      u.parity);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S>
hipError_t launch_diag_t(const StepArgs &a, const double *regions, double *partial, double *out, int nruns,
                         int parity)
{
    using C = typename Store<S>::C;
    const dim3 block(a.tx, a.ty);
    diag_partial_kernel<S><<<a.ntiles, block, 0, a.stream>>>(a.runs, a.tiles, static_cast<const S *>(a.f),
                                                               static_cast<const C *>(a.psi), regions,
                                                               partial, parity, a.xcd);
    diag_final_kernel<<<nruns, 256, 0, a.stream>>>(a.runs, partial, out);
    return hipGetLastError();
}

hipError_t launch_step(int precision, const StepArgs &a, int parity)
{
    switch (precision) {
    case PREC_FP64: return launch_step_t<double>(a, parity);
    case PREC_FP32: return launch_step_t<float>(a, parity);
    case PREC_BF16: return launch_step_t<bf16_t>(a, parity);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_collide(int precision, const StepArgs &a, int parity)
{
    switch (precision) {
    case PREC_FP64: return launch_collide_t<double>(a, parity);
    case PREC_FP32: return launch_collide_t<float>(a, parity);
    case PREC_BF16: return launch_collide_t<bf16_t>(a, parity);
    }
    return hipErrorInvalidValue;
}

// Plain 16-byte vector copy, grid-stride: the reference streaming kernel.
__global__ void __launch_bounds__(256) copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t stream)
{
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 256 * 64 ? (want > 0 ? want : 1) : 256 * 64);
    copy_kernel<<<blocks, 256, 0, stream>>>(static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    return hipGetLastError();
}

hipError_t launch_psi(int precision, const StepArgs &a, int parity)
{
    switch (precision) {
    case PREC_FP64: return launch_psi_t<double>(a, parity);
    case PREC_FP32: return launch_psi_t<float>(a, parity);
    case PREC_BF16: return launch_psi_t<bf16_t>(a, parity);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_util(int precision, const UtilArgs &u)
{
    switch (precision) {
    case PREC_FP64: return launch_util_t<double>(u);
    case PREC_FP32: return launch_util_t<float>(u);
    case PREC_BF16: return launch_util_t<bf16_t>(u);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_diag(int precision, const StepArgs &a, const double *regions, double *partial, double *out,
                       int nruns, int parity)
{
    switch (precision) {
    case PREC_FP64: return launch_diag_t<double>(a, regions, partial, out, nruns, parity);
    case PREC_FP32: return launch_diag_t<float>(a, regions, partial, out, nruns, parity);
    case PREC_BF16: return launch_diag_t<bf16_t>(a, regions, partial, out, nruns, parity);
    }
    return hipErrorInvalidValue;
}

} // namespace lbm
