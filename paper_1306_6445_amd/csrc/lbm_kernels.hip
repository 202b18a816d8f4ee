// HIP kernels (gfx950) of the D2Q9 pseudopotential MRT lattice Boltzmann step
// with the surface-tension source term of Li & Luo (arXiv:1306.6445).
//
// One step = two launches over the tile work list of every run in a context:
//   psi_kernel      rho = sum_a f_a (Eq. 6) -> psi(rho) (Section II, Eq. 23)
//   collide_kernel  psi tile + halo in LDS -> F (Eq. 7), Q (Eq. 19) -> v (Eq. 6)
//                   -> m = M f, m_eq (Eq. 3), S (Eqs. 5, 8), C (Eq. 18)
//                   -> m* (Eq. 17) -> f* = M^-1 m* -> in-place AA store (Eq. 4)
// or one launch of fused_kernel, which computes psi of the tile and its halo
// itself and writes the next state to a second buffer.  All are HBM-bound
// streaming kernels: one thread per node, nine coalesced structure-of-arrays
// loads and stores, moment transforms as add chains.
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
    int x, y, ld; // ld: row stride of the run's device arrays
    int64_t N;
    const Nbr *n;
    C ref;
    C *f;
    const float *rp;
    const float *rt;
    int LXr;
    template <int A> __device__ __forceinline__ void operator()()
    {
        const int64_t i = PARITY == 0 ? even_slot<A>(x, y, ld, N) : odd_slot<A>(x, y, *n, ld, N);
        C refA = ref;
        if constexpr (kWriterRef<S>) {
            if (rt)
                refA = C(rt[upwind_offset<A>(*n, LXr)]);
            else if (rp)
                refA = C(rp[upwind_node<A>(x, y, *n, ld)]);
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
    int x, y, ld;
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
        const int64_t i = PARITY == 0 ? even_slot<B>(x, y, ld, N) : odd_slot<B>(x, y, *n, ld, N);
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

// The same two for a node whose neighbours lie inside the grid (no periodic
// seam, no wall): every slot is a fixed offset from the node's flat index, and
// the writer density of f_a sits at x - e_a in the LDS tile rt.
template <typename S, int PARITY>
struct LoadPopsInner {
    using C = typename Store<S>::C;
    const S *fb;
    int64_t idx;
    int ld;
    int64_t N;
    C ref;
    C *f;
    const float *rt;
    int LXr;
    template <int A> __device__ __forceinline__ void operator()()
    {
        const int64_t i = PARITY == 0 ? (int64_t)A * N + idx : odd_slot_inner<A>(idx, ld, N);
        C refA = ref;
        if constexpr (kWriterRef<S>) refA = C(rt[-ey_of(A) * LXr - ex_of(A)]);
        f[A] = Store<S>::template load<A>(fb, i, refA);
    }
};

template <typename S, int PARITY>
struct StorePopsInner {
    using C = typename Store<S>::C;
    S *fb;
    int64_t idx;
    int ld;
    int64_t N;
    C ref;
    const C *f;
    bool sr;
    uint32_t hb;
    template <int A> __device__ __forceinline__ void operator()()
    {
        constexpr int B = opp_of(A);
        const int64_t i = PARITY == 0 ? (int64_t)B * N + idx : odd_slot_inner<B>(idx, ld, N);
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
__device__ __forceinline__ void load_node(const S *fb, int x, int y, int ld, int64_t N, const Nbr &n,
                                          typename Store<S>::C ref, typename Store<S>::C *f,
                                          const float *rp = nullptr, const float *rt = nullptr, int LXr = 0)
{
    LoadPops<S, PARITY> op{fb, x, y, ld, N, &n, ref, f, rp, rt, LXr};
    for9(op);
}

// The w x hgt block of a per-node array at (x0, y0) with an h-node halo into
// LDS (periodic wrap, clamp across walls), row stride w + 2h; every thread of
// the workgroup takes part.
template <typename T>
__device__ __forceinline__ void stage_tile(T *lds, const T *src, int x0, int y0, int w, int hgt, int h,
                                           const RunDev &r)
{
    const int LX = w + 2 * h, LY = hgt + 2 * h, nt = blockDim.x * blockDim.y;
    for (int i = threadIdx.y * blockDim.x + threadIdx.x; i < LX * LY; i += nt) {
        const int ly = i / LX, lx = i - ly * LX;
        const int gx = psi_coord(x0 - h + lx, r.nx, r.bc_x);
        const int gy = psi_coord(y0 - h + ly, r.ny, r.bc_y);
        lds[i] = src[(int64_t)gy * r.pitch + gx];
    }
}

// The workgroup's tile (blockDim.x x blockDim.y nodes) with an H-node halo.
template <typename T, int H = 1>
__device__ __forceinline__ void stage_halo_tile(T *lds, const T *src, const Tile &t, const RunDev &r)
{
    stage_tile<T>(lds, src, t.x0, t.y0, blockDim.x, blockDim.y, H, r);
}

template <typename S, int PARITY>
__device__ __forceinline__ void store_node(S *fb, int x, int y, int ld, int64_t N, const Nbr &n,
                                           typename Store<S>::C ref, const typename Store<S>::C *f,
                                           bool sr = false, uint32_t hb = 0)
{
    StorePops<S, PARITY> op{fb, x, y, ld, N, &n, ref, f, sr, hb};
    for9(op);
}

// Runtime-parity variants for the (non-hot) utility kernels.
template <typename S>
__device__ __forceinline__ void load_node_rt(const S *fb, int x, int y, int ld, int64_t N, const Nbr &n,
                                             typename Store<S>::C ref, typename Store<S>::C *f, int parity,
                                             const float *rp = nullptr)
{
    if (parity == 0)
        load_node<S, 0>(fb, x, y, ld, N, n, ref, f, rp);
    else
        load_node<S, 1>(fb, x, y, ld, N, n, ref, f, rp);
}

// Location of f_a(x) in the current state (put/get kernels); refv, when
// given, holds the base density of each direction (writer-referenced storage).
template <typename S, int PARITY>
struct PutPops {
    using C = typename Store<S>::C;
    S *fb;
    int x, y, ld;
    int64_t N;
    const Nbr *n;
    C ref;
    const C *f;
    const C *refv;
    template <int A> __device__ __forceinline__ void operator()()
    {
        const int64_t i = PARITY == 0 ? even_slot<A>(x, y, ld, N) : odd_slot<A>(x, y, *n, ld, N);
        Store<S>::template store<A>(fb, i, f[A], refv ? refv[A] : ref);
    }
};

template <typename S>
__device__ __forceinline__ void put_node_rt(S *fb, int x, int y, int ld, int64_t N, const Nbr &n,
                                            typename Store<S>::C ref, const typename Store<S>::C *f, int parity,
                                            const typename Store<S>::C *refv = nullptr)
{
    if (parity == 0) {
        PutPops<S, 0> op{fb, x, y, ld, N, &n, ref, f, refv};
        for9(op);
    } else {
        PutPops<S, 1> op{fb, x, y, ld, N, &n, ref, f, refv};
        for9(op);
    }
}

// f = M^-1 m for the orthogonal D2Q9 basis (rho, e, zeta, jx, qx, jy, qy, pxx, pxy):
// M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
// The conserved moments (rho, jx, jy) are not merely multiplied by a rounded
// reciprocal: 9 * fl(1/9) = 1 + 7.5e-9 in FP32, which would add mass at every
// step (1.5e-4 after 20,000 steps).  div_const corrects the product by its
// exact residual, which leaves no bias (the same mass drift as an IEEE
// division, at a third of the instructions).
template <typename C>
__device__ __forceinline__ void moments_to_pops(const C *m, C *f)
{
    const C a = div_const<C>(m[0], 9.0), b = m[1] * C(1.0 / 36.0), c = m[2] * C(1.0 / 36.0);
    const C d = div_const<C>(m[3], 6.0), e = m[4] * C(1.0 / 12.0), g = div_const<C>(m[5], 6.0);
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
// rho: the node's density, node_density(fv) (the collision conserves it).
template <typename C, bool MR = false>
__device__ __forceinline__ void collide_node(const RunDev &r, const C *fv, C rho, const C *lc, int LX, C *fs)
{
    const RunPar<C> &k = r.template par<C>();
    const C p0 = lc[0];
    const C p1 = lc[1], p3 = lc[-1], p2 = lc[LX], p4 = lc[-LX];
    const C p5 = lc[LX + 1], p6 = lc[LX - 1], p7 = lc[-LX - 1], p8 = lc[-LX + 1];

    const C G = k.G;
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
        const C G2 = k.G2;
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
    const C kq = k.kappa * G * C(0.5) * p0;
    const C Qxx = kq * (C(1.0 / 3.0) * (p1 + p3 - C(2) * p0) + C(1.0 / 12.0) * dsum);
    const C Qyy = kq * (C(1.0 / 3.0) * (p2 + p4 - C(2) * p0) + C(1.0 / 12.0) * dsum);
    const C Qxy = kq * (C(1.0 / 12.0) * ((p5 + p7) - (p6 + p8)));

    // Eq. (6): density (node_density, from the caller) and velocity (with F/2)
    const C sA = fv[1] + fv[3], sB = fv[2] + fv[4], sD = (fv[5] + fv[7]) + (fv[6] + fv[8]);
    const C d13 = fv[1] - fv[3], d24 = fv[2] - fv[4];
    const C d57 = fv[5] - fv[7], d86 = fv[8] - fv[6];
    const C jx = d13 + (d57 + d86);
    const C jy = d24 + (d57 - d86);
    const C irho = recip<C>(rho);
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
    const C S1 = C(6) * (vx * Fx + vy * Fy) + k.sig_coef * F2;
    const C S7 = C(2) * (vx * Fx - vy * Fy);
    const C S8 = vx * Fy + vy * Fx;
    // Eq. (18)
    const C trQ = Qxx + Qyy;
    // Section V.C: the viscosity steps from nu_V to nu_L at the threshold density
    const C se = k.s_e, sz = k.s_zeta, sq = k.s_q;
    const C sv = rho < k.rho_nu ? k.s_nu_low : k.s_nu;
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
}

// ----------------------------------------------------------- psi kernel

// psi of one node from its populations: the Eq. (6) density (node_density:
// compensated in FP32) and psi(rho) in the arithmetic type.  NaN and false
// where psi is not real.  rho_out receives the density.
template <typename C>
__device__ __forceinline__ bool node_psi(const RunDev &r, const C *fv, C &out, C &rho_out)
{
    const C rho = node_density<C>(fv);
    rho_out = rho;
    C ps;
    const bool ok = eval_psi<C>(r, rho, ps);
    out = ok ? ps : C(NAN);
    return ok;
}

template <typename S, int PARITY>
__global__ void __launch_bounds__(kMaxTileThreads) psi_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
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
    const int ld = r.pitch;
    const int64_t N = r.dstride;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    C fv[9];
    load_node<S, PARITY>(f + r.f_off, x, y, ld, N, n, r.template par<C>().rho_ref, fv, nullptr,
                         kWriterRef<S> ? rtile + (threadIdx.y + 1) * LXr + threadIdx.x + 1 : nullptr, LXr);
    C ps, rho;
    if (!node_psi<C>(r, fv, ps, rho)) status[t.run] = 1;
    psi[r.n_off + (int64_t)y * ld + x] = ps;
}

// ------------------------------------------------------- collide kernel

template <typename S, int PARITY, int H = 1>
__global__ void __launch_bounds__(kMaxTileThreads) collide_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
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
    const int ld = r.pitch;
    const int64_t N = r.dstride;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    const C ref = r.template par<C>().rho_ref;
    C fv[9];
    load_node<S, PARITY>(f + r.f_off, x, y, ld, N, n, ref, fv, nullptr,
                         kWriterRef<S> ? rtile + (threadIdx.y + H) * LX + threadIdx.x + H : nullptr, LX);

    // psi at x + e_a (and x + 2 e_a) from LDS
    const C *lc = lds + (threadIdx.y + H) * LX + (threadIdx.x + H);
    C fs[9];
    const C rho = node_density<C>(fv);
    collide_node<C, (H > 1)>(r, fv, rho, lc, LX, fs);
    if constexpr (kWriterRef<S>) {
        // base density of every population written here: this node's density,
        // kept for the readers of the next step
        const int64_t gi = r.n_off + (int64_t)y * ld + x;
        const uint32_t hb = fmix32((uint32_t)gi ^ fmix32(seed[PARITY]));
        store_node<S, PARITY>(f + r.f_off, x, y, ld, N, n, rho, fs, true, hb);
        rcur[gi] = (float)rho;
    } else {
        store_node<S, PARITY>(f + r.f_off, x, y, ld, N, n, ref, fs);
    }
}

// ---------------------------------------------------- fused step kernel
// One launch per step, out of place.  The state of parity p is read from one
// population buffer and the state of parity p ^ 1 is written to the other, at
// the addresses the in-place AA step would write, so every other routine
// reads either buffer with the same addressing.  Instead of a psi pass, a
// tile computes psi on its H-node halo from the halo nodes' own populations
// in the source buffer, which no workgroup of the launch writes.  Each
// population is then read from HBM once and written once per step; the halo
// rows come again from L2 (vertically adjacent tiles run under one L2, see
// work_index).  The densities, psi and the collision are the same arithmetic
// as psi_kernel + collide_kernel, so both schedules give the same bits.
// bf16 storage: the writer densities of the previous step are staged with an
// H + 1 halo (a halo node's populations decode with its upwind neighbours'
// densities), the rounding seed of the step is derived from the last one as
// the psi pass would, and the tile's own densities go to the next array.

// k-th cell of the H-node ring around a TX x TY tile in an LX x LY LDS
// tile: H full rows on top, H at the bottom, then H cells at each end of the
// TY rows between.  The ring has 2 H (LX + TY) cells.
__device__ __forceinline__ void ring_cell(int k, int TX, int LX, int LY, int H, int &lx, int &ly)
{
    const int rows = H * LX;
    if (k < 2 * rows) {
        const bool top = k < rows;
        const int j = top ? k : k - rows;
        const int q = j / LX;
        ly = top ? q : LY - H + q;
        lx = j - q * LX;
    } else {
        const int j = k - 2 * rows, w = 2 * H;
        const int q = j / w, c = j - q * w;
        ly = H + q;
        lx = c < H ? c : TX + c;
    }
}

// Index arithmetic of a tile of the fused step (the same addresses in each):
//   kInner     the tile, its halo ring and their upwind neighbours lie inside
//              the grid, so no node sits on a periodic seam or a wall and
//              every slot is a fixed offset from the node index;
//   kPeriodic  both axes of the run are periodic: wrapped neighbours, with
//              the wall tests of the streaming rule known false at compile time
//              (FP64 and FP32 storage; for bf16 the extra path costs more in
//              registers than it saves);
//   kGeneral   wrapped or clamped neighbours and per-node wall tests.
constexpr int kGeneral = 0, kPeriodic = 1, kInner = 2;

template <typename S, int PARITY, int H, int R, int MODE>
__device__ __forceinline__ void fused_tile(const RunDev &r, const Tile &t, const S *__restrict__ fin,
                                           S *__restrict__ fout, int32_t *__restrict__ status,
                                           typename Store<S>::C *lds, const float *rtile,
                                           float *__restrict__ rcur, uint32_t sd)
{
    using C = typename Store<S>::C;
    constexpr bool INNER = MODE == kInner;
    const int nx = r.nx, ny = r.ny, ld = r.pitch;
    const int bcx = MODE == kPeriodic ? BC_PERIODIC : r.bc_x, bcy = MODE == kPeriodic ? BC_PERIODIC : r.bc_y;
    const int TX = blockDim.x, TY = blockDim.y, TYR = R * TY;
    const int LX = TX + 2 * H, LY = TYR + 2 * H;
    const int64_t N = r.dstride;
    const C ref = r.template par<C>().rho_ref;
    const int LXr = LX + 2, ox = t.x0 - H - 1, oy = t.y0 - H - 1;
    // LDS cell of writer densities centred on a node seen at unwrapped (ux, uy):
    // across a wall the clamped node's own cell; on a periodic axis the
    // unwrapped cell, whose neighbours hold the wrapped neighbours' densities
    auto rcentre = [&](int ux, int uy, int gx, int gy) -> const float * {
        if constexpr (kWriterRef<S>)
            return rtile + ((bcy == BC_WALL ? gy : uy) - oy) * LXr + ((bcx == BC_WALL ? gx : ux) - ox);
        else
            return nullptr;
    };

    // this thread's nodes; past the grid edge (a partial tile) the thread
    // fills its LDS cell with the wrapped or clamped node and stores nothing
    const int x = t.x0 + threadIdx.x;
    const bool xin = INNER || x < nx;
    const int gx = xin ? x : psi_coord(x, nx, bcx);
    C fv[R][9];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int y = t.y0 + threadIdx.y + j * TY;
        if constexpr (INNER) {
            LoadPopsInner<S, PARITY> op{fin, (int64_t)y * ld + x, ld, N, ref, fv[j], rcentre(x, y, x, y), LXr};
            for9(op);
        } else {
            const int gy = y < ny ? y : psi_coord(y, ny, bcy);
            const Nbr n = neighbours(gx, gy, nx, ny, bcx, bcy);
            load_node<S, PARITY>(fin, gx, gy, ld, N, n, ref, fv[j], nullptr, rcentre(x, y, gx, gy), LXr);
        }
    }

    // psi of the halo ring (periodic wrap, clamp across walls, as in
    // stage_halo_tile), from the populations of the halo nodes
    bool bad = false;
    const int nring = 2 * H * (LX + TYR);
    for (int k = threadIdx.y * TX + threadIdx.x; k < nring; k += TX * TY) {
        int lx, ly;
        ring_cell(k, TX, LX, LY, H, lx, ly);
        const int ux = t.x0 - H + lx, uy = t.y0 - H + ly;
        C fh[9];
        if constexpr (INNER) {
            LoadPopsInner<S, PARITY> op{fin, (int64_t)uy * ld + ux, ld, N, ref, fh, rcentre(ux, uy, ux, uy), LXr};
            for9(op);
        } else {
            const int hx = psi_coord(ux, nx, bcx), hy = psi_coord(uy, ny, bcy);
            const Nbr nh = neighbours(hx, hy, nx, ny, bcx, bcy);
            load_node<S, PARITY>(fin, hx, hy, ld, N, nh, ref, fh, nullptr, rcentre(ux, uy, hx, hy), LXr);
        }
        C ph, rh;
        bad |= !node_psi<C>(r, fh, ph, rh);
        lds[ly * LX + lx] = ph;
    }
    C rv[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        C p0;
        bad |= !node_psi<C>(r, fv[j], p0, rv[j]);
        lds[(threadIdx.y + j * TY + H) * LX + threadIdx.x + H] = p0;
    }
    if (bad) status[t.run] = 1;
    __syncthreads();
    if (!xin) return;

#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int y = t.y0 + threadIdx.y + j * TY;
        if (!INNER && y >= ny) break;
        const C *lc = lds + (threadIdx.y + j * TY + H) * LX + (threadIdx.x + H);
        C fs[9];
        const C rho = rv[j];
        collide_node<C, (H > 1)>(r, fv[j], rho, lc, LX, fs);
        const int64_t idx = (int64_t)y * ld + x;
        // bf16 storage: this node's density is the base of what it writes
        // (as in collide_kernel), with stochastic rounding
        bool sr = false;
        uint32_t hb = 0;
        C base = ref;
        if constexpr (kWriterRef<S>) {
            const int64_t gi = r.n_off + idx;
            hb = fmix32((uint32_t)gi ^ fmix32(sd));
            sr = true;
            base = rho;
            rcur[gi] = (float)rho;
        }
        if constexpr (INNER) {
            StorePopsInner<S, PARITY> op{fout, idx, ld, N, base, fs, sr, hb};
            for9(op);
        } else {
            const Nbr n = neighbours(x, y, nx, ny, bcx, bcy);
            store_node<S, PARITY>(fout, x, y, ld, N, n, base, fs, sr, hb);
        }
    }
}

template <typename S, int PARITY, int H, int R>
__global__ void __launch_bounds__(kMaxTileThreads) fused_kernel(const RunDev *__restrict__ runs, const Tile *__restrict__ tiles,
                                                    const S *__restrict__ src, S *__restrict__ dst,
                                                    int32_t *__restrict__ status, int xcd,
                                                    const float *__restrict__ rprev, float *__restrict__ rcur,
                                                    uint32_t *__restrict__ seed)
{
    using C = typename Store<S>::C;
    extern __shared__ unsigned char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);

    // a tile of TX x (R TY) nodes: each thread takes R nodes, TY rows apart
    const Tile t = tiles[work_index(xcd)];
    const RunDev &r = runs[t.run];
    const int TX = blockDim.x, TYR = R * blockDim.y;
    const int LX = TX + 2 * H, LY = TYR + 2 * H;

    // bf16: writer densities of the previous step over the tile and an H + 1 halo
    float *rtile = reinterpret_cast<float *>(lds + LX * LY);
    uint32_t sd = 0;
    if constexpr (kWriterRef<S>) {
        // rounding seed of this step: one more than the last step's (the
        // value psi_kernel would write; no workgroup reads slot PARITY here)
        sd = seed[PARITY ^ 1] + 1u;
        if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) seed[PARITY] = sd;
        stage_tile<float>(rtile, rprev + r.n_off, t.x0, t.y0, TX, TYR, H + 1, r);
        __syncthreads();
    }
    // the same decision for every thread of the workgroup
    const bool inner = t.x0 - H - 1 >= 0 && t.x0 + TX + H + 1 <= r.nx && t.y0 - H - 1 >= 0 &&
                       t.y0 + TYR + H + 1 <= r.ny;
    if (inner)
        fused_tile<S, PARITY, H, R, kInner>(r, t, src + r.f_off, dst + r.f_off, status, lds, rtile, rcur, sd);
    else if (!kWriterRef<S> && r.bc_x == BC_PERIODIC && r.bc_y == BC_PERIODIC)
        fused_tile<S, PARITY, H, R, kPeriodic>(r, t, src + r.f_off, dst + r.f_off, status, lds, rtile, rcur, sd);
    else
        fused_tile<S, PARITY, H, R, kGeneral>(r, t, src + r.f_off, dst + r.f_off, status, lds, rtile, rcur, sd);
}

// ------------------------------------------------------- utility kernels
// These run once per call of the host API (initialisation, read-back,
// diagnostics); one thread per node of a single run.  Host-order arrays
// (staging, [k][ny][nx]) are indexed y nx + x; the run's device arrays
// y pitch + x.

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
        put_node_rt<S>(f + r.f_off, x, y, r.pitch, r.dstride, n, C(0), fc, parity, refv);
        rdec[r.n_off + (int64_t)y * r.pitch + x] = (float)rho[idx];
    } else {
        put_node_rt<S>(f + r.f_off, x, y, r.pitch, r.dstride, n, r.template par<C>().rho_ref, fc, parity);
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
    const int64_t N = (int64_t)r.nx * r.ny, Nd = r.dstride;
    C fc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fc[a] = (C)src[a * N + idx];
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    if constexpr (kWriterRef<S>) {
        C refv[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) refv[a] = (C)canonical_density(src, N, upwind_node_rt(a, x, y, n, r.nx));
        put_node_rt<S>(f + r.f_off, x, y, r.pitch, Nd, n, C(0), fc, parity, refv);
        rdec[r.n_off + (int64_t)y * r.pitch + x] = canonical_density(src, N, idx);
    } else {
        put_node_rt<S>(f + r.f_off, x, y, r.pitch, Nd, n, r.template par<C>().rho_ref, fc, parity);
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
    load_node_rt<S>(f + r.f_off, x, y, r.pitch, r.dstride, n, r.template par<C>().rho_ref, fc, parity,
                    rdec ? rdec + r.n_off : nullptr);
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
    const int nx = r.nx, ny = r.ny, ld = r.pitch;
    const int64_t N = r.dstride;
    const Nbr n = neighbours(x, y, nx, ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, ld, N, n, r.template par<C>().rho_ref, fc, parity, rdec ? rdec + r.n_off : nullptr);
    double fd[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fd[a] = (double)fc[a];
    rho = ((fd[0] + (fd[1] + fd[3])) + (fd[2] + fd[4])) + ((fd[5] + fd[7]) + (fd[6] + fd[8]));
    const double jx = (fd[1] - fd[3]) + ((fd[5] - fd[7]) + (fd[8] - fd[6]));
    const double jy = (fd[2] - fd[4]) + ((fd[5] - fd[7]) + (fd[6] - fd[8]));
    const C *pb = psi + r.n_off;
    auto P = [&](int dx, int dy) -> double {
        const int gx = psi_coord(x + dx, nx, r.bc_x), gy = psi_coord(y + dy, ny, r.bc_y);
        return (double)pb[(int64_t)gy * ld + gx];
    };
    const double p0 = P(0, 0);
    const double sx = (P(1, 0) - P(-1, 0)) / 3.0 + ((P(1, 1) - P(-1, -1)) + (P(1, -1) - P(-1, 1))) / 12.0;
    const double sy = (P(0, 1) - P(0, -1)) / 3.0 + ((P(1, 1) - P(-1, -1)) + (P(-1, 1) - P(1, -1))) / 12.0;
    double Fx = -r.pd.G * p0 * sx, Fy = -r.pd.G * p0 * sy;
    if (r.pd.G2 != 0.0) { // Eq. (9), second range
        const double tx = (P(2, 0) - P(-2, 0)) / 3.0 + ((P(2, 2) - P(-2, -2)) + (P(2, -2) - P(-2, 2))) / 12.0;
        const double ty = (P(0, 2) - P(0, -2)) / 3.0 + ((P(2, 2) - P(-2, -2)) + (P(-2, 2) - P(2, -2))) / 12.0;
        Fx += -r.pd.G2 * p0 * tx;
        Fy += -r.pd.G2 * p0 * ty;
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

// Bulk pressure p_EOS(rho) of every node of one run in FP64 (the pressure of
// the Laplace law, Section V.A; rho summed in FP64 from the stored state).
template <typename S>
__global__ void pressure_kernel(const RunDev *__restrict__ runs, int run, const S *__restrict__ f,
                                double *__restrict__ out, int parity, const float *__restrict__ rdec)
{
    using C = typename Store<S>::C;
    const RunDev &r = runs[run];
    int x, y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!node_of(r, idx, x, y)) return;
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, r.pitch, r.dstride, n, r.template par<C>().rho_ref, fc, parity,
                    rdec ? rdec + r.n_off : nullptr);
    double fd[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) fd[a] = (double)fc[a];
    const double rho = ((fd[0] + (fd[1] + fd[3])) + (fd[2] + fd[4])) + ((fd[5] + fd[7]) + (fd[6] + fd[8]));
    out[idx] = rho > 0.0 ? eval_pressure(r, rho) : NAN;
}

// Populations of a w x h window of one run at (x0, y0), FP64 [9][h][w]; the
// window's coordinates wrap on periodic axes (the host checks that it lies
// inside the grid on wall axes).
template <typename S>
__global__ void window_kernel(const RunDev *__restrict__ runs, int run, const S *__restrict__ f, int x0, int y0,
                              int w, int h, double *__restrict__ out, int parity, const float *__restrict__ rdec)
{
    using C = typename Store<S>::C;
    const RunDev &r = runs[run];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)w * h) return;
    const int j = (int)(k / w), i = (int)(k - (int64_t)j * w);
    const int x = psi_coord(x0 + i, r.nx, r.bc_x), y = psi_coord(y0 + j, r.ny, r.bc_y);
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, r.pitch, r.dstride, n, r.template par<C>().rho_ref, fc, parity,
                    rdec ? rdec + r.n_off : nullptr);
    const int64_t M = (int64_t)w * h;
#pragma unroll
    for (int a = 0; a < 9; ++a) out[a * M + k] = (double)fc[a];
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
    const int64_t N = r.dstride;
    const Nbr n = neighbours(x, y, r.nx, r.ny, r.bc_x, r.bc_y);
    C fc[9];
    load_node_rt<S>(f + r.f_off, x, y, r.pitch, N, n, r.template par<C>().rho_ref, fc, parity, rdec ? rdec + r.n_off : nullptr);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) s += (double)fc[a];
    out[y] = s;
}

// Droplet diagnostics: per-tile FP64 partial sums, then a per-run reduction.
// Partial layout (8 doubles): mass, sum rho_in, n_in, sum rho_out, n_out,
// sum p_in, sum p_out, max speed.
// the diagnostics run on the step's tiles: one thread per node, up to the
// largest tile
constexpr int DIAG_THREADS = kMaxTileThreads;

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

// One-run descriptor and tile work list written into device memory from
// kernel arguments (no host copy), and the run's status flag cleared: the
// tables of the context-free step (lbm_step_noalloc).
__global__ void table_setup_kernel(RunDev r, RunDev *__restrict__ runs, Tile *__restrict__ tiles, int ntx,
                                   int ntiles, int tx, int ty, int32_t *__restrict__ status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        runs[0] = r;
        status[0] = 0;
    }
    if (i < ntiles) tiles[i] = Tile{0, (i % ntx) * tx, (i / ntx) * ty, 0};
}

hipError_t launch_table_setup(const RunDev &r, RunDev *runs, Tile *tiles, int ntx, int ntiles, int tx, int ty,
                              int32_t *status, hipStream_t stream)
{
    const int bs = 256;
    table_setup_kernel<<<(ntiles + bs - 1) / bs, bs, 0, stream>>>(r, runs, tiles, ntx, ntiles, tx, ty, status);
    return hipGetLastError();
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

template <typename S, int H, int R>
hipError_t launch_fused_hr(const StepArgs &a, int parity)
{
    using C = typename Store<S>::C;
    const dim3 block(a.tx, a.ty);
    const int LX = a.tx + 2 * H, LY = R * a.ty + 2 * H;
    const uint32_t lds = sizeof(C) * LX * LY + (kWriterRef<S> ? sizeof(float) * (LX + 2) * (LY + 2) : 0);
    const S *src = static_cast<const S *>(a.f);
    S *dst = static_cast<S *>(a.f_alt);
    // parity p reads the writer densities R[p ^ 1] and writes R[p]
    const float *rprev = parity ? a.r0 : a.r1;
    float *rcur = parity ? a.r1 : a.r0;
    if (parity == 0)
        hipExtLaunchKernelGGL(fused_kernel<S, 0, H, R>, dim3(a.nftiles), block, lds, a.stream, a.ev_start,
                              a.ev_stop, 0, a.runs, a.ftiles, src, dst, a.status, a.xcd, rprev, rcur, a.seed);
    else
        hipExtLaunchKernelGGL(fused_kernel<S, 1, H, R>, dim3(a.nftiles), block, lds, a.stream, a.ev_start,
                              a.ev_stop, 0, a.runs, a.ftiles, src, dst, a.status, a.xcd, rprev, rcur, a.seed);
    return hipGetLastError();
}

template <typename S, int H>
hipError_t launch_fused_h(const StepArgs &a, int parity)
{
    switch (a.fused) {
    case 1: return launch_fused_hr<S, H, 1>(a, parity);
    case 2: return launch_fused_hr<S, H, 2>(a, parity);
    case 4: return launch_fused_hr<S, H, 4>(a, parity);
    }
    return hipErrorInvalidValue;
}

template <typename S>
hipError_t launch_fused_t(const StepArgs &a, int parity)
{
    if (!a.f_alt || !a.ftiles || (kWriterRef<S> && (!a.r0 || !a.r1 || !a.seed))) return hipErrorInvalidValue;
    return a.halo == 1 ? launch_fused_h<S, 1>(a, parity) : launch_fused_h<S, 2>(a, parity);
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
    case UTIL_PRESSURE:
        pressure_kernel<S><<<nb, bs, 0, u.stream>>>(u.runs, u.run, f, u.buf, u.parity, rdec);
        break;
    case UTIL_WINDOW:
        window_kernel<S><<<blocks_for((int64_t)u.ww * u.wh, bs), bs, 0, u.stream>>>(u.runs, u.run, f, u.wx0, u.wy0,
                                                                                  u.ww, u.wh, u.buf, u.parity, rdec);
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
