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

// Loads f_a(x) of the current state.  Base density: the per-run constant
// ref, or, for writer-referenced storage, the density of the node that wrote
// the slot, from an LDS tile of writer densities (rt, centred on x, row
// stride LXr) or from the run's array (rp).
template <typename S, int PARITY>
struct LoadPops {
    using C = typename Store<S>::C;
    const S *fb;
    int x, y, nx;
    int64_t N;
    const Nbr *n;
    C ref;
    C *f;
    const float *rp;
    const float *rt;
    int LXr;
    template <int A> __device__ __forceinline__ void operator()()
    {
        const int64_t i = PARITY == 0 ? even_slot<A>(x, y, nx, N) : odd_slot<A>(x, y, *n, nx, N);
        C refA = ref;
        if constexpr (kWriterRef<S>) {
            if (rt)
                refA = C(rt[upwind_offset<A>(*n, LXr)]);
            else if (rp)
                refA = C(rp[upwind_node<A>(x, y, *n, nx)]);
        }
        f[A] = Store<S>::template load<A>(fb, i, refA);
    }
};

// Stores f*_a(x).  With sr, bf16 rounding is stochastic: the node's hash hb
// seeds the 32-bit linear congruential generator of O'Neill's PCG family
// (multiplier 747796405, increment 2891336453), whose top 16 bits feed one
// direction per step of the generator.
template <typename S, int PARITY>
struct StorePops {
    using C = typename Store<S>::C;
    S *fb;
    int x, y, nx;
    int64_t N;
    const Nbr *n;
    C ref;
    const C *f;
    bool sr;
    uint32_t hb;
    template <int A> __device__ __forceinline__ void operator()()
    {
        constexpr int B = opp_of(A);
        // even step: f*_A goes to slot opp(A) of this node;
        // odd step: f*_A goes where the odd-state rule keeps f_opp(A) of this node.
        const int64_t i = PARITY == 0 ? even_slot<B>(x, y, nx, N) : odd_slot<B>(x, y, *n, nx, N);
        if constexpr (kWriterRef<S>) {
            if (sr) {
                hb = hb * 747796405u + 2891336453u;
                Store<S>::template store_sr<A>(fb, i, f[A], ref, hb >> 16);
                return;
            }
        }
        Store<S>::template store<A>(fb, i, f[A], ref);
    }
};

template <typename S, int PARITY>
__device__ __forceinline__ void load_node(const S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                          typename Store<S>::C ref, typename Store<S>::C *f,
                                          const float *rp = nullptr, const float *rt = nullptr, int LXr = 0)
{
    LoadPops<S, PARITY> op{fb, x, y, nx, N, &n, ref, f, rp, rt, LXr};
    for9(op);
}

// Tile of a per-node array with an H-node halo into LDS (periodic wrap, clamp
// across walls), row stride TX + 2H; every thread of the block takes part.
template <typename T, int H = 1>
__device__ __forceinline__ void stage_halo_tile(T *lds, const T *src, const Tile &t, const RunDev &r)
{
    const int TX = blockDim.x, TY = blockDim.y;
    const int LX = TX + 2 * H, LY = TY + 2 * H;
    for (int i = threadIdx.y * TX + threadIdx.x; i < LX * LY; i += TX * TY) {
        const int ly = i / LX, lx = i - ly * LX;
        const int gx = psi_coord(t.x0 - H + lx, r.nx, r.bc_x);
        const int gy = psi_coord(t.y0 - H + ly, r.ny, r.bc_y);
        lds[i] = src[(int64_t)gy * r.nx + gx];
    }
}

template <typename S, int PARITY>
__device__ __forceinline__ void store_node(S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                           typename Store<S>::C ref, const typename Store<S>::C *f,
                                           bool sr = false, uint32_t hb = 0)
{
    StorePops<S, PARITY> op{fb, x, y, nx, N, &n, ref, f, sr, hb};
    for9(op);
}

// Runtime-parity variants for the (non-hot) utility kernels.
template <typename S>
__device__ __forceinline__ void load_node_rt(const S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                             typename Store<S>::C ref, typename Store<S>::C *f, int parity,
                                             const float *rp = nullptr)
{
    if (parity == 0)
        load_node<S, 0>(fb, x, y, nx, N, n, ref, f, rp);
    else
        load_node<S, 1>(fb, x, y, nx, N, n, ref, f, rp);
}

// Location of f_a(x) in the current state (put/get kernels); refv, when
// given, holds the base density of each direction (writer-referenced storage).
template <typename S, int PARITY>
struct PutPops {
    using C = typename Store<S>::C;
    S *fb;
    int x, y, nx;
    int64_t N;
    const Nbr *n;
    C ref;
    const C *f;
    const C *refv;
    template <int A> __device__ __forceinline__ void operator()()
    {
        const int64_t i = PARITY == 0 ? even_slot<A>(x, y, nx, N) : odd_slot<A>(x, y, *n, nx, N);
        Store<S>::template store<A>(fb, i, f[A], refv ? refv[A] : ref);
    }
};

template <typename S>
__device__ __forceinline__ void put_node_rt(S *fb, int x, int y, int nx, int64_t N, const Nbr &n,
                                            typename Store<S>::C ref, const typename Store<S>::C *f, int parity,
                                            const typename Store<S>::C *refv = nullptr)
{
    if (parity == 0) {
        PutPops<S, 0> op{fb, x, y, nx, N, &n, ref, f, refv};
        for9(op);
    } else {
        PutPops<S, 1> op{fb, x, y, nx, N, &n, ref, f, refv};
        for9(op);
    }
}

// f = M^-1 m for the orthogonal D2Q9 basis (rho, e, zeta, jx, qx, jy, qy, pxx, pxy):
// M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
// The conserved moments (rho, jx, jy) are divided, not multiplied by a rounded
// reciprocal: 9 * fl(1/9) = 1 + 7.5e-9 in FP32, which would add mass at every
// step (1.5e-4 after 20,000 steps); a correctly rounded quotient has no bias.
template <typename C>
__device__ __forceinline__ void moments_to_pops(const C *m, C *f)
{
    const C a = m[0] / C(9), b = m[1] * C(1.0 / 36.0), c = m[2] * C(1.0 / 36.0);
    const C d = m[3] / C(6), e = m[4] * C(1.0 / 12.0), g = m[5] / C(6);
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

// One node's collision: psi(x + e_a) from an LDS tile (lc points at psi(x),
// rows LX apart) and the pre-collision populations fv -> post-collision fs.
// MR: the multi-range force of Eq. (9), which also reads psi(x + 2 e_a).
// Returns the density (which the collision conserves).
template <typename C, bool MR = false>
__device__ __forceinline__ C collide_node(const RunDev &r, const C *fv, const C *lc, int LX, C *fs)
{
    const C p0 = lc[0];
    const C p1 = lc[1], p3 = lc[-1], p2 = lc[LX], p4 = lc[-LX];
    const C p5 = lc[LX + 1], p6 = lc[LX - 1], p7 = lc[-LX - 1], p8 = lc[-LX + 1];

    const C G = C(r.G);
    // Eq. (7): F = -G psi(x) sum_a w_a psi(x + e_a) e_a, w = 1/3 (axis), 1/12 (diagonal)
    const C sx = C(1.0 / 3.0) * (p1 - p3) + C(1.0 / 12.0) * ((p5 - p7) + (p8 - p6));
    const C sy = C(1.0 / 3.0) * (p2 - p4) + C(1.0 / 12.0) * ((p5 - p7) + (p6 - p8));
    C Fx, Fy, F2; // F2 = |F|^2 / psi^2
    if constexpr (MR) {
        // Eq. (9): F = -psi(x) sum_a w_a [G1 psi(x + e_a) + G2 psi(x + 2 e_a)] e_a
        const int L2 = 2 * LX;
        const C q1 = lc[2], q3 = lc[-2], q2 = lc[L2], q4 = lc[-L2];
        const C q5 = lc[L2 + 2], q6 = lc[L2 - 2], q7 = lc[-L2 - 2], q8 = lc[-L2 + 2];
        const C tx = C(1.0 / 3.0) * (q1 - q3) + C(1.0 / 12.0) * ((q5 - q7) + (q8 - q6));
        const C ty = C(1.0 / 3.0) * (q2 - q4) + C(1.0 / 12.0) * ((q5 - q7) + (q6 - q8));
        const C G2 = C(r.G2);
        const C gx = G * sx + G2 * tx, gy = G * sy + G2 * ty;
        Fx = -p0 * gx;
        Fy = -p0 * gy;
        F2 = gx * gx + gy * gy;
    } else {
        Fx = -G * p0 * sx;
        Fy = -G * p0 * sy;
        F2 = G * G * (sx * sx + sy * sy);
    }
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
    // |F|^2 / psi^2 = G^2 (sx^2 + sy^2) exactly (Eq. 7; F2 above).
    const C S1 = C(6) * (vx * Fx + vy * Fy) + C(r.sig_coef) * F2;
    const C S7 = C(2) * (vx * Fx - vy * Fy);
    const C S8 = vx * Fy + vy * Fx;
    // Eq. (18)
    const C trQ = Qxx + Qyy;
    // Section V.C: the viscosity steps from nu_V to nu_L at the threshold density
    const C se = C(r.s_e), sz = C(r.s_zeta), sq = C(r.s_q);
    const C sv = rho < C(r.rho_nu) ? C(r.s_nu_low) : C(r.s_nu);
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

    moments_to_pops<C>(ms, fs);
    return rho;
}

// ----------------------------------------------------------- psi kernel

template <typename S, int PARITY>
__global__ void __launch_bounds__(256) psi_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                           const S *__restrict__ f, typename Store<S>::C *__restrict__ psi,
                           int32_t *__restrict__ status, int xcd, const float *__restrict__ rprev,
                           uint32_t *__restrict__ seed)
{
    using C = typename Store<S>::C;
    if constexpr (kWriterRef<S>) {
        // rounding seed of this step's collide launch: one more than the last
        // step's (writing it again for the same state gives the same value)
        if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) seed[PARITY] = seed[PARITY ^ 1] + 1u;
    }
    const Tile t = tiles[work_index(xcd)];
    const RunDev &r = runs[t.run];
    const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y;
    const int nx = r.nx, ny = r.ny;
    // writer densities of the tile and its halo (bf16 storage)
    extern __shared__ float rtile[];
    const int LXr = blockDim.x + 2;
    if constexpr (kWriterRef<S>) {
        stage_halo_tile<float>(rtile, rprev + r.n_off, t, r);
        __syncthreads();
    }
    if (x >= nx || y >= ny) return;
    const int64_t N = (int64_t)nx * ny;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    C fv[9];
    load_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, C(r.rho_ref), fv, nullptr,
                         kWriterRef<S> ? rtile + (threadIdx.y + 1) * LXr + threadIdx.x + 1 : nullptr, LXr);
    // Eq. (6): rho = sum_a f_a, and psi(rho): both in FP64 whatever the storage
    // (a handful of operations per node in a memory-bound kernel; in FP32 the
    // rounding of the EOS biases the vapour density the interface settles to)
    double fd[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fd[a] = (double)fv[a];
    const double rho = ((fd[0] + (fd[1] + fd[3])) + (fd[2] + fd[4])) + ((fd[5] + fd[7]) + (fd[6] + fd[8]));
    double ps;
    if (!eval_psi<double>(r, rho, ps)) {
        status[t.run] = 1;
        ps = NAN;
    }
    psi[r.n_off + (int64_t)y * nx + x] = (C)ps;
}

// ------------------------------------------------------- collide kernel

template <typename S, int PARITY, int H = 1>
__global__ void __launch_bounds__(256) collide_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                               S *__restrict__ f, const typename Store<S>::C *__restrict__ psi, int xcd,
                               const float *__restrict__ rprev, float *__restrict__ rcur,
                               const uint32_t *__restrict__ seed)
{
    using C = typename Store<S>::C;
    extern __shared__ unsigned char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);

    const Tile t = tiles[work_index(xcd)];
    const RunDev &r = runs[t.run];
    const int nx = r.nx, ny = r.ny;
    const int TX = blockDim.x, TY = blockDim.y;
    const int LX = TX + 2 * H, LY = TY + 2 * H;
    const C *pb = psi + r.n_off;

    // psi of the tile plus an H-node halo (H = 2 for the multi-range force of
    // Eq. 9), wrapped or clamped per boundary (and, for bf16 storage, the
    // writer densities of the same cells)
    stage_halo_tile<C, H>(lds, pb, t, r);
    float *rtile = reinterpret_cast<float *>(lds + LX * LY);
    if constexpr (kWriterRef<S>) stage_halo_tile<float, H>(rtile, rprev + r.n_off, t, r);
    __syncthreads();

    const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int64_t N = (int64_t)nx * ny;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    const C ref = C(r.rho_ref);
    C fv[9];
    load_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, ref, fv, nullptr,
                         kWriterRef<S> ? rtile + (threadIdx.y + H) * LX + threadIdx.x + H : nullptr, LX);

    // psi at x + e_a (and x + 2 e_a) from LDS
    const C *lc = lds + (threadIdx.y + H) * LX + (threadIdx.x + H);
    C fs[9];
    const C rho = collide_node<C, (H > 1)>(r, fv, lc, LX, fs);
    if constexpr (kWriterRef<S>) {
        // base density of every population written here: this node's density,
        // kept for the readers of the next step
        const int64_t gi = r.n_off + (int64_t)y * nx + x;
        const uint32_t hb = fmix32((uint32_t)gi ^ fmix32(seed[PARITY]));
        store_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, rho, fs, true, hb);
        rcur[gi] = (float)rho;
    } else {
        store_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, ref, fs);
    }
}

// ---------------------------------------------------- fused step kernel
// One launch per step.  One wavefront owns a tile of 64 x RY nodes (origin
// x0, y0; w x h nodes inside the grid) and an array E_T of (64+2) x (RY+2)
// density partial sums: cell (lx, ly) stands for the node at unwrapped
// coordinates (x0-1+lx, y0-1+ly) and holds the sum of the populations that
// reach that node at the next step from nodes of T (Eq. 4, halfway
// bounce-back included).  Interior cells therefore hold complete densities;
// edge and halo cells hold T's share.  A step of tile T:
//   A. density of every node of T and its one-node halo = sum, in a fixed
//      order, of the E cells of the tiles whose extended region covers the
//      node; psi(rho) into LDS (Section II, Eq. 23);
//   B. row by row: collide (Eqs. 6, 7, 19, 3, 5, 8, 18, 17), AA-store, and
//      scatter f* into next-step densities: x +- 1 by lane shifts, y +- 1 by a
//      three-row window in registers; the two halo columns go through LDS.
// E arrays are double-buffered by step parity.
constexpr int kFusedTX = 64;

// Tiles whose extended region covers coordinate g along one axis: their tile
// index along the axis and g's local cell in them, in the order (lower
// neighbour, owner, upper neighbour).  Periodic axes wrap; walls end the row.
struct Cover {
    int c[3], l[3];
    bool v[3];
};

template <int T>
__device__ __forceinline__ Cover cover_axis(int g, int n, int ntiles, int bc)
{
    Cover cv;
    const int cO = g / T, off = g - cO * T;
    const int wO = min(T, n - cO * T);
    cv.v[0] = cv.v[2] = false;
    cv.c[1] = cO;
    cv.l[1] = off + 1;
    cv.v[1] = true;
    cv.c[0] = cv.l[0] = cv.c[2] = cv.l[2] = 0;
    if (off == 0 && (bc == BC_PERIODIC || cO > 0)) {
        const int cL = cO == 0 ? ntiles - 1 : cO - 1;
        cv.c[0] = cL;
        cv.l[0] = min(T, n - cL * T) + 1; // upper halo cell of the lower neighbour
        cv.v[0] = true;
    }
    if (off == wO - 1 && (bc == BC_PERIODIC || cO < ntiles - 1)) {
        cv.c[2] = cO == ntiles - 1 ? 0 : cO + 1;
        cv.l[2] = 0; // lower halo cell of the upper neighbour
        cv.v[2] = true;
    }
    return cv;
}

template <typename C, int RY>
__device__ __forceinline__ C gather_rho(const C *__restrict__ e_run, int gx, int gy, int nx, int ny, int tiles_x,
                                        int tiles_y, int bcx, int bcy)
{
    constexpr int LX = kFusedTX + 2, NC = LX * (RY + 2);
    const Cover cx = cover_axis<kFusedTX>(gx, nx, tiles_x, bcx);
    const Cover cy = cover_axis<RY>(gy, ny, tiles_y, bcy);
    C s = C(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (!cy.v[j]) continue;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (!cx.v[i]) continue;
            s += e_run[(int64_t)(cy.c[j] * tiles_x + cx.c[i]) * NC + cy.l[j] * LX + cx.l[i]];
        }
    }
    return s;
}

// value of v held by lane - 1 (0 in lane 0) / lane + 1 (0 in lane 63)
template <typename C> __device__ __forceinline__ C from_left(C v)
{
    const C u = __shfl_up(v, 1, 64);
    return __lane_id() == 0 ? C(0) : u;
}
template <typename C> __device__ __forceinline__ C from_right(C v)
{
    const C u = __shfl_down(v, 1, 64);
    return __lane_id() == 63 ? C(0) : u;
}

template <typename S, int PARITY, int RY>
__global__ void __launch_bounds__(kFusedTX)
fused_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, S *__restrict__ f,
             const typename Store<S>::C *__restrict__ e_in, typename Store<S>::C *__restrict__ e_out,
             int32_t *__restrict__ status, int xcd)
{
    using C = typename Store<S>::C;
    constexpr int LX = kFusedTX + 2, LY = RY + 2, NC = LX * LY;
    __shared__ C psi[LY * LX];
    __shared__ C ring[2][LY]; // next-step shares of the left / right halo columns

    const int lane = threadIdx.x;
    const int wi = work_index(xcd);
    const Tile t = tiles[wi];
    const RunDev &r = runs[t.run];
    const int nx = r.nx, ny = r.ny, bcx = r.bc_x, bcy = r.bc_y;
    const int tiles_x = (nx + kFusedTX - 1) / kFusedTX, tiles_y = (ny + RY - 1) / RY;
    const int w = min(kFusedTX, nx - t.x0), h = min(RY, ny - t.y0);
    const C *e_run = e_in + (int64_t)r.ftile_begin * NC;
    const C *e_own = e_in + (int64_t)wi * NC;

    // the first row's populations are fetched while the densities are gathered
    const int x = t.x0 + lane;
    const bool active = lane < w;
    const int64_t N = (int64_t)nx * ny;
    const C ref = C(r.rho_ref);
    C fnext[9];
    if (active) {
        const Nbr n = neighbours(x, t.y0, nx, ny, bcx, bcy);
        load_node<S, PARITY>(f + r.f_off, x, t.y0, nx, N, n, ref, fnext);
    }

    // A. densities of the tile and its halo, then psi; every lane issues all
    // of its gathers before the first use
    constexpr int J = (NC + kFusedTX - 1) / kFusedTX;
    C rho[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int i = lane + j * kFusedTX;
        const int ly = i / LX, lx = i - ly * LX;
        rho[j] = C(1);
        if (i < NC) {
            if (lx >= 2 && lx < w && ly >= 2 && ly < h) {
                rho[j] = e_own[i]; // inside the tile, away from its edges: this tile's cell is complete
            } else {
                const int gx = psi_coord(t.x0 - 1 + lx, nx, bcx);
                const int gy = psi_coord(t.y0 - 1 + ly, ny, bcy);
                rho[j] = gather_rho<C, RY>(e_run, gx, gy, nx, ny, tiles_x, tiles_y, bcx, bcy);
            }
        }
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int i = lane + j * kFusedTX;
        if (i < NC) {
            double ps; // the EOS in FP64 whatever the storage, as in psi_kernel
            if (!eval_psi<double>(r, (double)rho[j], ps)) {
                bad = true;
                ps = NAN;
            }
            psi[i] = (C)ps;
        }
    }
    if (bad) status[t.run] = 1;
    if (lane < LY) {
        ring[0][lane] = C(0);
        ring[1][lane] = C(0);
    }
    __syncthreads();

    // B. rows of the tile.  Row k + 1 is fetched before row k is stored: the
    // AA addresses of different nodes never coincide, so the order is free.
    C *eo = e_out + (int64_t)wi * NC;
    C r0_prev = C(0), up_prev = C(0), up_prev2 = C(0);
    for (int k = 0; k < h; ++k) {
        const int y = t.y0 + k;
        C fs[9];
        if (active) {
            C fv[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) fv[a] = fnext[a];
            if (k + 1 < h) {
                const Nbr n1 = neighbours(x, y + 1, nx, ny, bcx, bcy);
                load_node<S, PARITY>(f + r.f_off, x, y + 1, nx, N, n1, ref, fnext);
            }
            const Nbr n = neighbours(x, y, nx, ny, bcx, bcy);
            collide_node<C>(r, fv, psi + (k + 1) * LX + (lane + 1), LX, fs);
            store_node<S, PARITY>(f + r.f_off, x, y, nx, N, n, ref, fs);
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a) fs[a] = C(0);
        }
        // populations whose destination lies beyond a wall come back to this node
        const bool wxm = bcx == BC_WALL && x == 0, wxp = bcx == BC_WALL && x == nx - 1;
        const bool wym = bcy == BC_WALL && y == 0, wyp = bcy == BC_WALL && y == ny - 1;
        C g[9], own = C(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int ex = ex_of(a), ey = ey_of(a);
            const bool wall = (ex > 0 && wxp) || (ex < 0 && wxm) || (ey > 0 && wyp) || (ey < 0 && wym);
            g[a] = wall ? C(0) : fs[a];
            own += wall ? fs[a] : C(0);
        }
        // shares of rows k (same row), k + 1 (up) and k - 1 (down) at this column
        const C r0 = (fs[0] + own) + from_left(g[1]) + from_right(g[3]);
        const C up = g[2] + from_left(g[5]) + from_right(g[6]);
        const C dn = g[4] + from_left(g[8]) + from_right(g[7]);
        if (lane == 0) { // left halo column, LDS row of node row k is k + 1
            ring[0][k] += g[7];
            ring[0][k + 1] += g[3];
            ring[0][k + 2] += g[6];
        }
        if (lane == w - 1) {
            ring[1][k] += g[8];
            ring[1][k + 1] += g[1];
            ring[1][k + 2] += g[5];
        }
        if (active) eo[k * LX + lane + 1] = k == 0 ? dn : (r0_prev + up_prev2) + dn;
        up_prev2 = up_prev;
        up_prev = up;
        r0_prev = r0;
    }
    if (active) {
        eo[h * LX + lane + 1] = r0_prev + up_prev2;
        eo[(h + 1) * LX + lane + 1] = up_prev;
    }
    __syncthreads();
    if (lane < h + 2) {
        eo[lane * LX] = ring[0][lane];
        eo[lane * LX + w + 1] = ring[1][lane];
    }
}

// E arrays of the current state: interior cells of every tile get the density
// of their node, halo cells 0 (so that the gather of the next step sums to rho).
template <typename S, int RY>
__global__ void __launch_bounds__(kFusedTX)
erho_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, const S *__restrict__ f,
            typename Store<S>::C *__restrict__ e_out, int parity)
{
    using C = typename Store<S>::C;
    constexpr int LX = kFusedTX + 2, LY = RY + 2, NC = LX * LY;
    const int wi = blockIdx.x;
    const Tile t = tiles[wi];
    const RunDev &r = runs[t.run];
    const int nx = r.nx, ny = r.ny;
    const int64_t N = (int64_t)nx * ny;
    C *eo = e_out + (int64_t)wi * NC;
    for (int i = threadIdx.x; i < NC; i += kFusedTX) {
        const int ly = i / LX, lx = i - ly * LX;
        const int x = t.x0 - 1 + lx, y = t.y0 - 1 + ly;
        C rho = C(0);
        if (lx >= 1 && lx <= kFusedTX && ly >= 1 && ly <= RY && x < nx && y < ny) {
            const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
            C fv[9];
            load_node_rt<S>(f + r.f_off, x, y, nx, N, n, C(r.rho_ref), fv, parity);
            rho = ((fv[0] + (fv[1] + fv[3])) + (fv[2] + fv[4])) + ((fv[5] + fv[7]) + (fv[6] + fv[8]));
        }
        eo[i] = rho;
    }
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
// Writer-referenced storage takes the initial density of each population's
// upwind node as its base and records the initial densities in rdec, the
// array the next step reads.
template <typename S>
__global__ void init_kernel(const RunDev *__restrict__ runs, int run, S *__restrict__ f,
                            const double *__restrict__ rho, const double *__restrict__ ux,
                            const double *__restrict__ uy, int parity, float *__restrict__ rdec)
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
    if constexpr (kWriterRef<S>) {
        C refv[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) refv[a] = (C)(float)rho[upwind_node_rt(a, x, y, n, r.nx)];
        put_node_rt<S>(f + r.f_off, x, y, r.nx, (int64_t)r.nx * r.ny, n, C(0), fc, parity, refv);
        rdec[r.n_off + idx] = (float)rho[idx];
    } else {
        put_node_rt<S>(f + r.f_off, x, y, r.nx, (int64_t)r.nx * r.ny, n, C(r.rho_ref), fc, parity);
    }
}

// Density of node k from canonical populations src[9][N], in FP64 summed in a
// fixed order, rounded to FP32 (the writer density of the storage).
__device__ __forceinline__ float canonical_density(const double *src, int64_t N, int64_t k)
{
    return (float)(((src[k] + (src[N + k] + src[3 * N + k])) + (src[2 * N + k] + src[4 * N + k])) +
                   ((src[5 * N + k] + src[7 * N + k]) + (src[6 * N + k] + src[8 * N + k])));
}

// Canonical FP64 populations [9][ny][nx] -> storage at the current parity.
// Writer-referenced storage: each node's own density becomes the base of the
// populations its neighbours read from it (rdec).
template <typename S>
__global__ void put_kernel(const RunDev *__restrict__ runs, int run, S *__restrict__ f,
                           const double *__restrict__ src, int parity, float *__restrict__ rdec)
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
    if constexpr (kWriterRef<S>) {
        C refv[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) refv[a] = (C)canonical_density(src, N, upwind_node_rt(a, x, y, n, r.nx));
        put_node_rt<S>(f + r.f_off, x, y, r.nx, N, n, C(0), fc, parity, refv);
        rdec[r.n_off + idx] = canonical_density(src, N, idx);
    } else {
        put_node_rt<S>(f + r.f_off, x, y, r.nx, N, n, C(r.rho_ref), fc, parity);
    }
}

// Storage at the current parity -> canonical FP64 populations [9][ny][nx].
template <typename S>
__global__ void get_kernel(const RunDev *__restrict__ runs, int run, const S *__restrict__ f,
                           double *__restrict__ dst, int parity, const float *__restrict__ rdec)
{
    using C = typename Store<S>::C;
    const RunDev &r = runs[run];
    int x, y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!node_of(r, idx, x, y)) return;
    const int64_t N = (int64_t)r.nx * r.ny;
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, r.nx, N, n, C(r.rho_ref), fc, parity, rdec ? rdec + r.n_off : nullptr);
#pragma unroll
    for (int a = 0; a < 9; ++a) dst[a * N + idx] = (double)fc[a];
}

// Density and Eq. (6) velocity of one run in FP64, using psi of the current state.
template <typename S>
__device__ __forceinline__ void node_macro(const RunDev &r, const S *f, const typename Store<S>::C *psi,
                                           int x, int y, int parity, const float *rdec, double &rho, double &vx,
                                           double &vy)
{
    using C = typename Store<S>::C;
    const int nx = r.nx, ny = r.ny;
    const int64_t N = (int64_t)nx * ny;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, nx, N, n, C(r.rho_ref), fc, parity, rdec ? rdec + r.n_off : nullptr);
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
    double Fx = -r.G * p0 * sx, Fy = -r.G * p0 * sy;
    if (r.G2 != 0.0) { // Eq. (9), second range
        const double tx = (P(2, 0) - P(-2, 0)) / 3.0 + ((P(2, 2) - P(-2, -2)) + (P(2, -2) - P(-2, 2))) / 12.0;
        const double ty = (P(0, 2) - P(0, -2)) / 3.0 + ((P(2, 2) - P(-2, -2)) + (P(-2, 2) - P(2, -2))) / 12.0;
        Fx += -r.G2 * p0 * tx;
        Fy += -r.G2 * p0 * ty;
    }
    vx = (jx + 0.5 * Fx) / rho;
    vy = (jy + 0.5 * Fy) / rho;
}

template <typename S>
__global__ void moments_kernel(const RunDev *__restrict__ runs, int run, const S *__restrict__ f,
                               const typename Store<S>::C *__restrict__ psi, double *__restrict__ out,
                               int parity, const float *__restrict__ rdec)
{
    const RunDev &r = runs[run];
    int x, y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!node_of(r, idx, x, y)) return;
    double rho, vx, vy;
    node_macro<S>(r, f, psi, x, y, parity, rdec, rho, vx, vy);
    const int64_t N = (int64_t)r.nx * r.ny;
    out[idx] = rho;
    out[N + idx] = vx;
    out[2 * N + idx] = vy;
}

// Density of one column x of a run in FP64 (interface tracking).
template <typename S>
__global__ void column_kernel(const RunDev *__restrict__ runs, int run, const S *__restrict__ f, int x,
                              double *__restrict__ out, int parity, const float *__restrict__ rdec)
{
    using C = typename Store<S>::C;
    const RunDev &r = runs[run];
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= r.ny) return;
    const int64_t N = (int64_t)r.nx * r.ny;
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, r.nx, N, n, C(r.rho_ref), fc, parity, rdec ? rdec + r.n_off : nullptr);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) s += (double)fc[a];
    out[y] = s;
}

// Droplet diagnostics: per-tile FP64 partial sums, then a per-run reduction.
// Partial layout (8 doubles): mass, sum rho_in, n_in, sum rho_out, n_out,
// sum p_in, sum p_out, max speed.
constexpr int DIAG_THREADS = 256;

template <typename S>
__global__ void __launch_bounds__(DIAG_THREADS)
diag_partial_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles, const S *__restrict__ f,
                    const typename Store<S>::C *__restrict__ psi, const double *__restrict__ regions,
                    double *__restrict__ partial, int parity, int xcd, const float *__restrict__ rdec)
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
        node_macro<S>(r, f, psi, x, y, parity, rdec, rho, vx, vy);
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
    // a step of parity p reads the writer densities R[p ^ 1]
    const float *rprev = parity ? a.r0 : a.r1;
    const uint32_t lds = kWriterRef<S> ? sizeof(float) * (a.tx + 2) * (a.ty + 2) : 0;
    if (parity == 0)
        hipExtLaunchKernelGGL(psi_kernel<S, 0>, dim3(a.ntiles), block, lds, a.stream, a.ev_start, a.ev_stop, 0,
                              a.runs, a.tiles, (const S *)f, psi, a.status, a.xcd, rprev, a.seed);
    else
        hipExtLaunchKernelGGL(psi_kernel<S, 1>, dim3(a.ntiles), block, lds, a.stream, a.ev_start, a.ev_stop, 0,
                              a.runs, a.tiles, (const S *)f, psi, a.status, a.xcd, rprev, a.seed);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_collide_t(const StepArgs &a, int parity)
{
    using C = typename Store<S>::C;
    const dim3 block(a.tx, a.ty);
    const int H = a.halo;
    const uint32_t lds = (sizeof(C) + (kWriterRef<S> ? sizeof(float) : 0)) * (a.tx + 2 * H) * (a.ty + 2 * H);
    S *f = static_cast<S *>(a.f);
    const C *psi = static_cast<const C *>(a.psi);
    // parity p reads R[p ^ 1], writes R[p]
    const float *rprev = parity ? a.r0 : a.r1;
    float *rcur = parity ? a.r1 : a.r0;
    const uint32_t *seed = a.seed;
    if (H == 1) {
        if (parity == 0)
            hipExtLaunchKernelGGL(collide_kernel<S, 0, 1>, dim3(a.ntiles), block, lds, a.stream, a.ev_start,
                                  a.ev_stop, 0, a.runs, a.tiles, f, psi, a.xcd, rprev, rcur, seed);
        else
            hipExtLaunchKernelGGL(collide_kernel<S, 1, 1>, dim3(a.ntiles), block, lds, a.stream, a.ev_start,
                                  a.ev_stop, 0, a.runs, a.tiles, f, psi, a.xcd, rprev, rcur, seed);
    } else {
        if (parity == 0)
            hipExtLaunchKernelGGL(collide_kernel<S, 0, 2>, dim3(a.ntiles), block, lds, a.stream, a.ev_start,
                                  a.ev_stop, 0, a.runs, a.tiles, f, psi, a.xcd, rprev, rcur, seed);
        else
            hipExtLaunchKernelGGL(collide_kernel<S, 1, 2>, dim3(a.ntiles), block, lds, a.stream, a.ev_start,
                                  a.ev_stop, 0, a.runs, a.tiles, f, psi, a.xcd, rprev, rcur, seed);
    }
    return hipGetLastError();
}

template <typename S, int RY>
hipError_t launch_fused_ry(const StepArgs &a, int parity)
{
    using C = typename Store<S>::C;
    S *f = static_cast<S *>(a.f);
    const C *ein = static_cast<const C *>(parity == 0 ? a.e0 : a.e1);
    C *eout = static_cast<C *>(parity == 0 ? a.e1 : a.e0);
    if (parity == 0)
        hipExtLaunchKernelGGL(fused_kernel<S, 0, RY>, dim3(a.nftiles), dim3(kFusedTX), 0, a.stream, a.ev_start,
                              a.ev_stop, 0, a.runs, a.ftiles, f, ein, eout, a.status, a.xcd);
    else
        hipExtLaunchKernelGGL(fused_kernel<S, 1, RY>, dim3(a.nftiles), dim3(kFusedTX), 0, a.stream, a.ev_start,
                              a.ev_stop, 0, a.runs, a.ftiles, f, ein, eout, a.status, a.xcd);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_fused_t(const StepArgs &a, int parity)
{
    switch (a.fused) {
    case 4: return launch_fused_ry<S, 4>(a, parity);
    case 8: return launch_fused_ry<S, 8>(a, parity);
    case 16: return launch_fused_ry<S, 16>(a, parity);
    }
    return hipErrorInvalidValue;
}

template <typename S>
hipError_t launch_erho_t(const StepArgs &a, int parity)
{
    using C = typename Store<S>::C;
    const S *f = static_cast<const S *>(a.f);
    C *e = static_cast<C *>(parity == 0 ? a.e0 : a.e1);
    switch (a.fused) {
    case 4: erho_kernel<S, 4><<<a.nftiles, kFusedTX, 0, a.stream>>>(a.runs, a.ftiles, f, e, parity); break;
    case 8: erho_kernel<S, 8><<<a.nftiles, kFusedTX, 0, a.stream>>>(a.runs, a.ftiles, f, e, parity); break;
    case 16: erho_kernel<S, 16><<<a.nftiles, kFusedTX, 0, a.stream>>>(a.runs, a.ftiles, f, e, parity); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S>
hipError_t launch_step_t(const StepArgs &a, int parity)
{
    StepArgs b = a;
    b.ev_start = b.ev_stop = nullptr;
    if (a.fused) return launch_fused_t<S>(b, parity);
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
    // writer densities of the current state (parity p): R[p ^ 1]
    float *rdec = u.parity ? u.r0 : u.r1;
    switch (u.op) {
    case UTIL_INIT:
        init_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, u.buf, u.ux, u.uy, u.parity, rdec);
        break;
    case UTIL_PUT:
        put_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, u.buf, u.parity, rdec);
        break;
    case UTIL_GET:
        get_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, u.buf, u.parity, rdec);
        break;
    case UTIL_COLUMN:
        column_kernel<S><<<blocks_for(u.nodes, bs), bs, 0, u.stream>>>(u.runs, u.run, f, u.index, u.buf, u.parity,
                                                                       rdec);
        break;
    case UTIL_MOMENTS:
        moments_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, static_cast<const C *>(u.psi), u.buf,
                                                      u.parity, rdec);
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
                                                               partial, parity, a.xcd,
                                                               parity ? a.r0 : a.r1);
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

hipError_t launch_fused(int precision, const StepArgs &a, int parity)
{
    switch (precision) {
    case PREC_FP64: return launch_fused_t<double>(a, parity);
    case PREC_FP32: return launch_fused_t<float>(a, parity);
    case PREC_BF16: return launch_fused_t<bf16_t>(a, parity);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_erho(int precision, const StepArgs &a, int parity)
{
    switch (precision) {
    case PREC_FP64: return launch_erho_t<double>(a, parity);
    case PREC_FP32: return launch_erho_t<float>(a, parity);
    case PREC_BF16: return launch_erho_t<bf16_t>(a, parity);
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

// Reference streaming kernel: a copy of 16-byte vectors, four independent
// non-temporal loads per thread before the four stores (two streams; on
// MI355X this form moves about 6.1 TB/s over 2 GiB, against about 4.6 TB/s
// for a one-vector grid-stride loop).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, int64_t n)
{
    const int64_t b = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b + 256 * k;
        if (i < n) v[k] = __builtin_nontemporal_load(&src[i]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b + 256 * k;
        if (i < n) __builtin_nontemporal_store(v[k], &dst[i]);
    }
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t stream)
{
    const int64_t n = (int64_t)(bytes / 16);
    const unsigned blocks = (unsigned)((n + 1023) / 1024);
    copy_kernel<<<blocks > 0 ? blocks : 1, 256, 0, stream>>>(static_cast<const u32x4 *>(src),
                                                            static_cast<u32x4 *>(dst), n);
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
