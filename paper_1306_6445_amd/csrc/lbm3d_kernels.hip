// HIP kernels (gfx950) of the D3Q19 extension of the pseudopotential MRT step
// with the surface-tension source term (Li & Luo, arXiv:1306.6445, Section VI
// names 3D as future work; the 3D form follows the derivation in the design
// notes).  One step is either one launch of fused3_kernel (psi of each plane
// computed in LDS while the tile marches along z; the default) or two
// launches over the nodes of one run:
//   psi3_kernel      rho = sum_a f_a (Eq. 6) -> psi(rho) (Section II; Eq. 23)
//   collide3_kernel  psi at the 18 neighbours -> F (Eq. 7) and Q (Eq. 19) with
//                    the weights 1/6, 1/12 -> v (Eq. 6) -> m = M f -> m_eq, S
//                    (M F_Guo), C = Lambda M df((3/5) tr Q I - Q + 2 sigma
//                    |F|^2/psi^2 I) -> m* (Eq. 17) -> f* = M^-1 m* -> stored
//                    at the node in the second population buffer.
// A buffer holds the post-collision state: slot a of node y is f*_a(y) of the
// last collision.  Streaming (Eq. 4) happens as the state is read: f_a(x) =
// f*_a(x - e_a), or f*_opp(a)(x) where x - e_a lies beyond a wall (halfway
// bounce-back).  Every slot is read once per step, so reads are shifted by
// one node and writes are aligned, which streams faster on this memory system
// than aligned reads with shifted writes.
// The moment transforms are the integer D3Q19 basis unrolled at compile time
// (zero entries dropped, +-1 entries as plain additions).
#include <hip/hip_ext.h>

#include "lbm3d_kernels.hpp"

namespace lbm3 {

using lbm::RunDev;
using lbm::RunPar;

__host__ __device__ constexpr int c2of(int a) { return ex3(a) * ex3(a) + ey3(a) * ey3(a) + ez3(a) * ez3(a); }
// equilibrium weights (the FP32 storage's rest-state deviations) and interaction weights
__host__ __device__ constexpr double w_eq3(int a) { return c2of(a) == 0 ? 1.0 / 3.0 : (c2of(a) == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr double w_int3(int a) { return c2of(a) == 0 ? 0.0 : (c2of(a) == 1 ? 1.0 / 6.0 : 1.0 / 12.0); }

// Orthogonal moment basis (rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx,
// pww, piww, pxy, pyz, pxz, mx, my, mz): row k at velocity a, and row norms.
__host__ __device__ constexpr int mrow(int k, int a)
{
    const int x = ex3(a), y = ey3(a), z = ez3(a), c2 = c2of(a);
    switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return x * (y * y - z * z);
    case 17: return y * (z * z - x * x);
    default: return z * (x * x - y * y);
    }
}
__host__ __device__ constexpr int mnorm(int k)
{
    return k == 0 ? 19 : k == 1 ? 2394 : k == 2 ? 252 : k <= 8 ? (k % 2 ? 10 : 40)
         : k == 9 ? 36 : k == 10 ? 72 : k == 11 ? 12 : k == 12 ? 24 : k <= 15 ? 4 : 8;
}

// sum_a c_a v_a over a < A with compile-time integer coefficients c_a = coef(a)
template <typename C, typename Coef, int A> struct IntDot {
    __device__ __forceinline__ static C run(const C *v)
    {
        const C rest = IntDot<C, Coef, A - 1>::run(v);
        constexpr int c = Coef::at(A - 1);
        if constexpr (c == 0)
            return rest;
        else if constexpr (c == 1)
            return rest + v[A - 1];
        else if constexpr (c == -1)
            return rest - v[A - 1];
        else
            return rest + C(c) * v[A - 1];
    }
};
template <typename C, typename Coef> struct IntDot<C, Coef, 0> {
    __device__ __forceinline__ static C run(const C *) { return C(0); }
};
template <int K> struct RowOf {
    __host__ __device__ static constexpr int at(int a) { return mrow(K, a); }
};
template <int A> struct ColOf {
    __host__ __device__ static constexpr int at(int k) { return mrow(k, A); }
};

template <typename C, int K> struct ToMoments {
    __device__ __forceinline__ static void run(const C *f, C *m)
    {
        ToMoments<C, K - 1>::run(f, m);
        m[K - 1] = IntDot<C, RowOf<K - 1>, 19>::run(f);
    }
};
template <typename C> struct ToMoments<C, 0> {
    __device__ __forceinline__ static void run(const C *, C *) {}
};

// f = M^-1 m = M^T diag(1 / norm) m: scale once, then integer columns
template <typename C, int A> struct ToPops {
    __device__ __forceinline__ static void run(const C *ms, C *f)
    {
        ToPops<C, A - 1>::run(ms, f);
        f[A - 1] = IntDot<C, ColOf<A - 1>, 19>::run(ms);
    }
};
template <typename C> struct ToPops<C, 0> {
    __device__ __forceinline__ static void run(const C *, C *) {}
};

template <typename C> __device__ __forceinline__ C rate(const Run3 &r, int k)
{
    if constexpr (std::is_same<C, float>::value)
        return r.sf[k];
    else
        return r.s[k];
}

template <typename C> __device__ __forceinline__ C two_sigma(const Run3 &r)
{
    if constexpr (std::is_same<C, float>::value)
        return r.sig2f;
    else
        return r.sig2;
}

// Storage: FP64 populations, or FP32 deviations f_a - w_a rho_ref.
template <typename S> __device__ __forceinline__ typename std::conditional<std::is_same<S, double>::value, double, float>::type
dec(S v, int a, float ref)
{
    if constexpr (std::is_same<S, double>::value)
        return v;
    else
        return v + (float)w_eq3(a) * ref;
}
template <typename S, typename C> __device__ __forceinline__ S enc(C v, int a, float ref)
{
    if constexpr (std::is_same<S, double>::value)
        return v;
    else
        return v - (float)w_eq3(a) * ref;
}

// Eq. (6) density of 19 populations: FP64 plain sum in velocity order; FP32
// every addition made error-free by Knuth's TwoSum, the errors added once.
template <typename C> __device__ __forceinline__ C density19(const C *f)
{
    if constexpr (std::is_same<C, float>::value) {
        float s = f[0], e = 0.f;
#pragma unroll
        for (int a = 1; a < 19; ++a) {
            float ea;
            s = lbm::two_sum(s, f[a], ea);
            e += ea;
        }
        return s + e;
    } else {
        C s = f[0];
#pragma unroll
        for (int a = 1; a < 19; ++a) s += f[a];
        return s;
    }
}

__device__ __forceinline__ void coords(const Run3 &r, int64_t n, int &x, int &y, int &z)
{
    const int nx = r.r.nx, ny = r.r.ny;
    const int64_t xy = (int64_t)nx * ny;
    z = (int)(n / xy);
    const int64_t rem = n - (int64_t)z * xy;
    y = (int)(rem / nx);
    x = (int)(rem - (int64_t)y * nx);
}

__device__ __forceinline__ int64_t node_at(const Run3 &r, int x, int y, int z)
{
    return ((int64_t)z * r.r.ny + y) * r.r.nx + x;
}

// Index of the slot that holds f_a(x) of the current state (pull_slot3); the
// same map places a state given as f_a(x) into a buffer.
__device__ __forceinline__ int64_t slot3(const Run3 &r, int64_t n, const AxisNb &X, const AxisNb &Y, const AxisNb &Z,
                                         int a)
{
    return pull_slot3(n, X, Y, Z, a, r.dstride);
}

template <typename S>
__device__ __forceinline__ void gather19(const Run3 &r, const S *__restrict__ f, int64_t n, const AxisNb &X,
                                         const AxisNb &Y, const AxisNb &Z,
                                         typename std::conditional<std::is_same<S, double>::value, double, float>::type *fv)
{
    const float ref = r.r.pf.rho_ref;
#pragma unroll
    for (int a = 0; a < 19; ++a) fv[a] = dec<S>(f[slot3(r, n, X, Y, Z, a)], a, ref);
}

// The same read for a buffer of less than 4 GiB (W32): every slot's byte
// offset from the buffer's start then fits in 32 bits, so each load takes one
// offset register beside the buffer's scalar base (64-bit addresses for all
// 19 loads in flight cost the fused kernel a wave per SIMD).  Offsets wrap
// modulo 2^32 and the final offset is exact.
struct AxisNb32 {
    uint32_t m, p;
    bool wm, wp;
};
__device__ __forceinline__ AxisNb32 narrow(const AxisNb &A) { return {(uint32_t)A.m, (uint32_t)A.p, A.wm, A.wp}; }
__device__ __forceinline__ uint32_t nb_off(const AxisNb32 &A, int e) { return e > 0 ? A.p : (e < 0 ? A.m : 0u); }
__device__ __forceinline__ bool nb_wall(const AxisNb32 &A, int e) { return e > 0 ? A.wp : (e < 0 && A.wm); }

template <typename S, typename Nb>
__device__ __forceinline__ void gather19_w32(const Run3 &r, const S *__restrict__ f, uint32_t n, const Nb &X,
                                             const Nb &Y, const AxisNb32 &Z,
                                             typename std::conditional<std::is_same<S, double>::value, double, float>::type *fv)
{
    const float ref = r.r.pf.rho_ref;
    const char *base = reinterpret_cast<const char *>(f);
    const uint32_t ds = (uint32_t)r.dstride;
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        const bool wall = nb_wall(X, -ex3(a)) || nb_wall(Y, -ey3(a)) || nb_wall(Z, -ez3(a));
        const uint32_t off = (uint32_t)nb_off(X, -ex3(a)) + (uint32_t)nb_off(Y, -ey3(a)) + nb_off(Z, -ez3(a));
        const uint32_t i = wall ? (uint32_t)opp3(a) * ds + n : (uint32_t)a * ds + n + off;
        fv[a] = dec<S>(*reinterpret_cast<const S *>(base + (uint32_t)(i * (uint32_t)sizeof(S))), a, ref);
    }
}

// neighbour offsets of the node n of a run
struct Nb3 {
    AxisNb X, Y, Z;
};
__device__ __forceinline__ Nb3 nb3_of(const Run3 &r, int64_t n)
{
    int x, y, z;
    coords(r, n, x, y, z);
    const int64_t sxy = (int64_t)r.r.nx * r.r.ny;
    return {axis_nb(x, r.r.nx, r.r.bc_x, 1), axis_nb(y, r.r.ny, r.r.bc_y, r.r.nx), axis_nb(z, r.nz, r.bc_z, sxy)};
}

template <typename S>
__global__ void __launch_bounds__(kThreads3) psi3_kernel(const Run3 *__restrict__ runs, const S *__restrict__ f,
                                                         void *__restrict__ psi_out, int32_t *__restrict__ status)
{
    using C = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
    const Run3 &r = runs[0];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= r.nodes) return;
    C fv[19];
    const Nb3 nb = nb3_of(r, n);
    gather19<S>(r, f, n, nb.X, nb.Y, nb.Z, fv);
    const C rho = density19<C>(fv);
    C ps;
    const bool ok = lbm::eval_psi<C>(r.r, rho, ps);
    if (!ok) status[0] = 1;
    static_cast<C *>(psi_out)[n] = ok ? ps : C(NAN);
}

// the "second-order" part of a moment vector for a symmetric tensor T
// (xx, yy, zz, xy, yz, xz): rows e, eps, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz
template <typename C> struct Second {
    C e, eps, pxx, pixx, pww, piww, pxy, pyz, pxz;
    __device__ __forceinline__ Second(C xx, C yy, C zz, C xy, C yz, C xz)
    {
        const C tr = xx + yy + zz;
        e = C(19) * tr;
        eps = C(-5.5) * tr;
        pxx = C(3) * xx - tr;
        pixx = C(-0.5) * pxx;
        pww = yy - zz;
        piww = C(-0.5) * pww;
        pxy = xy;
        pyz = yz;
        pxz = xz;
    }
};

// One node's collision, shared by both schedules: psi_at(a) gives psi at
// x + e_a (a = 0: the node itself; beyond a wall, the adjacent fluid node), fv
// holds the node's 19 populations of the current state (streamed), n its
// index.  The same source expressions in both kernels give the same bits.
template <typename S, typename C, bool W32, typename PsiAt>
__device__ __forceinline__ void collide3(const Run3 &r, S *__restrict__ fout, const C *fv, int64_t n,
                                         const PsiAt &psi_at)
{
    // Eq. (7) and Eq. (19) with the 3D weights; psi beyond a wall = psi of the adjacent fluid node
    const RunPar<C> &k = r.r.template par<C>();
    const C p0 = psi_at(0);
    C sx = 0, sy = 0, sz = 0, qxx = 0, qyy = 0, qzz = 0, qxy = 0, qyz = 0, qxz = 0;
#pragma unroll
    for (int a = 1; a < 19; ++a) {
        const C pa = psi_at(a);
        const C w = C(w_int3(a));
        if (ex3(a)) sx += C(ex3(a)) * w * pa;
        if (ey3(a)) sy += C(ey3(a)) * w * pa;
        if (ez3(a)) sz += C(ez3(a)) * w * pa;
        const C d = w * (pa - p0);
        if (ex3(a)) qxx += d;
        if (ey3(a)) qyy += d;
        if (ez3(a)) qzz += d;
        if (ex3(a) * ey3(a)) qxy += C(ex3(a) * ey3(a)) * d;
        if (ey3(a) * ez3(a)) qyz += C(ey3(a) * ez3(a)) * d;
        if (ex3(a) * ez3(a)) qxz += C(ex3(a) * ez3(a)) * d;
    }
    const C G = k.G;
    const C Fx = -G * p0 * sx, Fy = -G * p0 * sy, Fz = -G * p0 * sz;
    const C F2 = G * G * (sx * sx + sy * sy + sz * sz); // |F|^2 / psi^2
    const C kq = k.kappa * G * C(0.5) * p0;
    qxx *= kq, qyy *= kq, qzz *= kq, qxy *= kq, qyz *= kq, qxz *= kq;

    C m[19];
    const C rho = density19<C>(fv);
    ToMoments<C, 19>::run(fv, m);
    // Eq. (6) velocity
    const C irho = lbm::recip<C>(rho);
    const C vx = (m[3] + C(0.5) * Fx) * irho, vy = (m[5] + C(0.5) * Fy) * irho, vz = (m[7] + C(0.5) * Fz) * irho;
    // equilibrium (tensor rho v v), Guo forcing (v F + F v) and flux shift
    // ((3/5) tr Q I - Q + 2 sigma |F|^2/psi^2 I) moments
    const Second<C> E2(rho * vx * vx, rho * vy * vy, rho * vz * vz, rho * vx * vy, rho * vy * vz, rho * vx * vz);
    const Second<C> S2(C(2) * vx * Fx, C(2) * vy * Fy, C(2) * vz * Fz, vx * Fy + vy * Fx, vy * Fz + vz * Fy,
                       vx * Fz + vz * Fx);
    const C iso = C(0.6) * (qxx + qyy + qzz) + two_sigma<C>(r) * F2;
    const Second<C> D2(iso - qxx, iso - qyy, iso - qzz, -qxy, -qyz, -qxz);
    C meq[19], Sm[19], Cm[19];
    meq[1] = C(-11) * rho + E2.e, Sm[1] = S2.e, Cm[1] = D2.e;
    meq[2] = C(3) * rho + E2.eps, Sm[2] = S2.eps, Cm[2] = D2.eps;
    meq[4] = C(-2.0 / 3.0) * rho * vx, Sm[4] = C(-2.0 / 3.0) * Fx, Cm[4] = 0;
    meq[6] = C(-2.0 / 3.0) * rho * vy, Sm[6] = C(-2.0 / 3.0) * Fy, Cm[6] = 0;
    meq[8] = C(-2.0 / 3.0) * rho * vz, Sm[8] = C(-2.0 / 3.0) * Fz, Cm[8] = 0;
    meq[9] = E2.pxx, Sm[9] = S2.pxx, Cm[9] = D2.pxx;
    meq[10] = E2.pixx, Sm[10] = S2.pixx, Cm[10] = D2.pixx;
    meq[11] = E2.pww, Sm[11] = S2.pww, Cm[11] = D2.pww;
    meq[12] = E2.piww, Sm[12] = S2.piww, Cm[12] = D2.piww;
    meq[13] = E2.pxy, Sm[13] = S2.pxy, Cm[13] = D2.pxy;
    meq[14] = E2.pyz, Sm[14] = S2.pyz, Cm[14] = D2.pyz;
    meq[15] = E2.pxz, Sm[15] = S2.pxz, Cm[15] = D2.pxz;
    meq[16] = meq[17] = meq[18] = 0, Sm[16] = Sm[17] = Sm[18] = 0, Cm[16] = Cm[17] = Cm[18] = 0;
    // Eq. (17); conserved moments: rho* = rho, and with the Eq. (6) velocity
    // j* = j - s_j (j - rho v) + (1 - s_j/2) F = j + F for any s_j
    C ms[19];
    ms[0] = rho;
    ms[3] = m[3] + Fx;
    ms[5] = m[5] + Fy;
    ms[7] = m[7] + Fz;
#pragma unroll
    for (int q = 1; q < 19; ++q) {
        if (q == 3 || q == 5 || q == 7) continue;
        const C s = rate<C>(r, q);
        ms[q] = m[q] - s * (m[q] - meq[q]) + (C(1) - C(0.5) * s) * Sm[q] + s * Cm[q];
    }
    // M^-1 = M^T diag(1 / norm): the conserved moments through div_const (in
    // FP32 the product with a rounded 1/19 or 1/10 would bias the mass and
    // momentum by an ulp every step; the FMA residual correction removes it)
#pragma unroll
    for (int q = 0; q < 19; ++q)
        ms[q] = (q == 0 || q == 3 || q == 5 || q == 7) ? lbm::div_const<C>(ms[q], (double)mnorm(q))
                                                      : ms[q] * C(1.0 / mnorm(q));
    C fs[19];
    ToPops<C, 19>::run(ms, fs);

    // f* stays at the node; the next read streams it (Eq. 4)
    const float ref = r.r.pf.rho_ref;
    if constexpr (W32) {
        char *base = reinterpret_cast<char *>(fout);
        const uint32_t ds = (uint32_t)r.dstride, n32 = (uint32_t)n;
#pragma unroll
        for (int a = 0; a < 19; ++a)
            *reinterpret_cast<S *>(base + (uint32_t)(((uint32_t)a * ds + n32) * (uint32_t)sizeof(S))) =
                enc<S, C>(fs[a], a, ref);
    } else {
#pragma unroll
        for (int a = 0; a < 19; ++a) fout[(int64_t)a * r.dstride + n] = enc<S, C>(fs[a], a, ref);
    }
}


// The collide pass runs over tiles of 2^txs x (256 >> txs) nodes in x-y, one
// z-plane each; the 1D work index decomposes with workgroup-uniform integer
// arithmetic, so no thread divides.  Workgroups reach the XCDs round-robin;
// work_index gives each XCD a contiguous range of tiles, so the neighbours
// whose gathers share cache lines (x), and whose psi rows and planes a tile
// reads (y, z), run under the same L2.
template <typename S>
__global__ void __launch_bounds__(kThreads3) collide3_kernel(const Run3 *__restrict__ runs, const S *__restrict__ fin,
                                                             S *__restrict__ fout, const void *__restrict__ psi_in,
                                                             int txs)
{
    using C = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
    const Run3 &r = runs[0];
    const int nx = r.r.nx, ny = r.r.ny, nz = r.nz, bcx = r.r.bc_x, bcy = r.r.bc_y, bcz = r.bc_z;
    int x, y, z;
    if (!collide3_node((unsigned)lbm::work_index(1), threadIdx.x, nx, ny, nz, txs, x, y, z)) return;
    const int64_t sxy = (int64_t)nx * ny;
    const int64_t n = (int64_t)z * sxy + (int64_t)y * nx + x;
    const AxisNb X = axis_nb(x, nx, bcx, 1), Y = axis_nb(y, ny, bcy, nx), Z = axis_nb(z, nz, bcz, sxy);
    const C *psi = static_cast<const C *>(psi_in);
    C fv[19];
    gather19<S>(r, fin, n, X, Y, Z, fv);
    collide3<S, C, false>(r, fout, fv, n, [&](int a) {
        return psi[n + nb_off(X, ex3(a)) + nb_off(Y, ey3(a)) + nb_off(Z, ez3(a))];
    });
}

// The fused step: one launch, psi computed where it is needed.  A workgroup
// owns an x-y tile of TX x TY nodes and marches along z through a chunk of
// planes.  psi of the plane ahead (the tile and a one-node ring around it; the
// ring and any tile column beyond the grid take the wrapped or clamped node)
// goes into one of four rotating LDS planes; after one barrier the tile's
// nodes of the current plane collide with the psi of planes z - 1, z, z + 1
// and store into the other buffer.  Each node's populations are gathered once
// (streamed from planes z, z + 1, z + 2 of the source), for its psi, and kept
// in registers until its collision one plane later; the ring's populations are
// re-read from cache.  Four slots let one barrier per
// plane suffice: the slot a plane's psi goes into was last read two planes
// earlier, before the previous barrier.  Out of place, so every workgroup
// reads only the unmodified source buffer.
template <typename S, int TX, int TY, bool W32>
__global__ void __launch_bounds__(TX * TY, (W32 && sizeof(S) == 4) ? 4 : 1) fused3_kernel(const Run3 *__restrict__ runs, const S *__restrict__ fin,
                                                         S *__restrict__ fout, int32_t *__restrict__ status, int zc)
{
    using C = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
    constexpr int PX = TX + 2, PY = TY + 2, PLANE = PX * PY, NT = TX * TY;
    static_assert(PLANE - NT <= NT, "one ring node per thread at most");
    __shared__ C lps[4][PLANE];
    const Run3 &r = runs[0];
    const int nx = r.r.nx, ny = r.r.ny, nz = r.nz, bcx = r.r.bc_x, bcy = r.r.bc_y, bcz = r.bc_z;
    const Fused3Thread q = fused3_thread((unsigned)lbm::work_index(1), threadIdx.x, nx, ny, nz, bcx, bcy, zc, TX, TY);
    const int x = q.x, y = q.y, cell = q.cell, rcell = q.rcell;
    const bool ring = q.ring;
    const int64_t col = q.col, rcol = q.rcol, sxy = (int64_t)nx * ny;
    // neighbour offsets of the column whose populations the thread gathers
    const AxisNb X = axis_nb(q.cx, nx, bcx, 1), Y = axis_nb(q.cy, ny, bcy, nx);

    bool bad = false;
    // psi of plane zl (wrapped or clamped) into its LDS slot; the thread's own
    // populations of that plane are left in fv
    auto psi_plane = [&](int zl, C *fv) {
        const int zw = lbm::psi_coord(zl, nz, bcz);
        const int64_t base = (int64_t)zw * sxy;
        const AxisNb Z = axis_nb(zw, nz, bcz, sxy);
        if constexpr (W32)
            gather19_w32<S>(r, fin, (uint32_t)base + (uint32_t)col, narrow(axis_nb(q.cx, nx, bcx, 1)),
                            narrow(axis_nb(q.cy, ny, bcy, nx)), narrow(Z), fv);
        else
            gather19<S>(r, fin, base + col, X, Y, Z, fv);
        C ps;
        bool ok = lbm::eval_psi<C>(r.r, density19<C>(fv), ps);
        lps[zl & 3][cell] = ok ? ps : C(NAN);
        bad |= !ok;
        if (ring) {
            C fr[19];
            if constexpr (W32)
                gather19_w32<S>(r, fin, (uint32_t)base + (uint32_t)rcol, narrow(axis_nb(q.rcx, nx, bcx, 1)),
                                narrow(axis_nb(q.rcy, ny, bcy, nx)), narrow(Z), fr);
            else
                gather19<S>(r, fin, base + rcol, axis_nb(q.rcx, nx, bcx, 1), axis_nb(q.rcy, ny, bcy, nx), Z, fr);
            ok = lbm::eval_psi<C>(r.r, density19<C>(fr), ps);
            lps[zl & 3][rcell] = ok ? ps : C(NAN);
            bad |= !ok;
        }
    };
    C fc[19], fn[19];
    psi_plane(q.z0 - 1, fn);
    psi_plane(q.z0, fc);
    for (int z = q.z0; z < q.z1; ++z) {
        psi_plane(z + 1, fn);
        __syncthreads();
        if (q.active) {
            const int64_t n = (int64_t)z * sxy + (int64_t)y * nx + x;
            collide3<S, C, W32>(r, fout, fc, n,
                                [&](int a) { return lps[(z + ez3(a)) & 3][cell + ey3(a) * PX + ex3(a)]; });
        }
#pragma unroll
        for (int a = 0; a < 19; ++a) fc[a] = fn[a];
    }
    if (bad) status[0] = 1;
}

// ------------------------------------------------------------- utilities

template <typename S>
__global__ void util3_kernel(const Run3 *__restrict__ runs, int op, const S *__restrict__ fin, S *__restrict__ fout,
                             const void *__restrict__ psi_in, double *__restrict__ buf)
{
    using C = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
    const Run3 &r = runs[0];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = r.nodes;
    if (n >= N) return;
    const float ref = r.r.pf.rho_ref;
    const Nb3 nb = nb3_of(r, n);
    if (op == 0) {
        C fv[19];
        gather19<S>(r, fin, n, nb.X, nb.Y, nb.Z, fv);
#pragma unroll
        for (int a = 0; a < 19; ++a) buf[a * N + n] = (double)fv[a];
    } else if (op == 2) {
        // f_a(x) into the slot it is read from (each slot written once)
#pragma unroll
        for (int a = 0; a < 19; ++a) fout[slot3(r, n, nb.X, nb.Y, nb.Z, a)] = enc<S, C>((C)buf[a * N + n], a, ref);
    } else if (op == 3) {
        const double rho = buf[n], v[3] = {buf[N + n], buf[2 * N + n], buf[3 * N + n]};
        const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
#pragma unroll
        for (int a = 0; a < 19; ++a) {
            const double eu = ex3(a) * v[0] + ey3(a) * v[1] + ez3(a) * v[2];
            const double fe = w_eq3(a) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * v2);
            fout[slot3(r, n, nb.X, nb.Y, nb.Z, a)] = enc<S, C>((C)fe, a, ref);
        }
    } else {
        // density and Eq. (6) velocity in FP64 from psi of the same state
        const C *psi = static_cast<const C *>(psi_in);
        C fv[19];
        gather19<S>(r, fin, n, nb.X, nb.Y, nb.Z, fv);
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 19; ++a) {
            rho += (double)fv[a];
            j[0] += ex3(a) * (double)fv[a];
            j[1] += ey3(a) * (double)fv[a];
            j[2] += ez3(a) * (double)fv[a];
        }
        int x, y, z;
        coords(r, n, x, y, z);
        double s[3] = {0.0, 0.0, 0.0};
        for (int a = 1; a < 19; ++a) {
            const int gx = lbm::psi_coord(x + ex3(a), r.r.nx, r.r.bc_x), gy = lbm::psi_coord(y + ey3(a), r.r.ny, r.r.bc_y),
                      gz = lbm::psi_coord(z + ez3(a), r.nz, r.bc_z);
            const double pa = (double)psi[node_at(r, gx, gy, gz)];
            s[0] += w_int3(a) * pa * ex3(a);
            s[1] += w_int3(a) * pa * ey3(a);
            s[2] += w_int3(a) * pa * ez3(a);
        }
        const double p0 = (double)psi[n], G = r.r.pd.G;
        buf[n] = rho;
        for (int i = 0; i < 3; ++i) buf[(i + 1) * N + n] = (j[i] - 0.5 * G * p0 * s[i]) / rho;
    }
}

template <typename S>
__global__ void __launch_bounds__(kThreads3) diag3_kernel(const Run3 *__restrict__ runs, const S *__restrict__ f,
                                                          const void *__restrict__ psi_in, int dims, double cx,
                                                          double cy, double cz, double r_in, double r_out,
                                                          double *__restrict__ partial)
{
    using C = typename std::conditional<std::is_same<S, double>::value, double, float>::type;
    __shared__ double red[8][kThreads3];
    const Run3 &r = runs[0];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tid = threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (n < r.nodes) {
        const C *psi = static_cast<const C *>(psi_in);
        C fv[19];
        const Nb3 nb = nb3_of(r, n);
        gather19<S>(r, f, n, nb.X, nb.Y, nb.Z, fv);
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 19; ++a) {
            rho += (double)fv[a];
            j[0] += ex3(a) * (double)fv[a];
            j[1] += ey3(a) * (double)fv[a];
            j[2] += ez3(a) * (double)fv[a];
        }
        int x, y, z;
        coords(r, n, x, y, z);
        double s[3] = {0.0, 0.0, 0.0};
        for (int a = 1; a < 19; ++a) {
            const int gx = lbm::psi_coord(x + ex3(a), r.r.nx, r.r.bc_x), gy = lbm::psi_coord(y + ey3(a), r.r.ny, r.r.bc_y),
                      gz = lbm::psi_coord(z + ez3(a), r.nz, r.bc_z);
            const double pa = (double)psi[node_at(r, gx, gy, gz)];
            s[0] += w_int3(a) * pa * ex3(a);
            s[1] += w_int3(a) * pa * ey3(a);
            s[2] += w_int3(a) * pa * ez3(a);
        }
        const double p0 = (double)psi[n], G = r.r.pd.G;
        double sp2 = 0.0;
        for (int i = 0; i < 3; ++i) {
            const double u = (j[i] - 0.5 * G * p0 * s[i]) / rho;
            sp2 += u * u;
        }
        // minimum-image distance on periodic axes; dims 2: a cylinder along z
        double dx = x - cx, dy = y - cy, dz = dims == 3 ? z - cz : 0.0;
        if (r.r.bc_x == lbm::BC_PERIODIC) dx -= r.r.nx * rint(dx / r.r.nx);
        if (r.r.bc_y == lbm::BC_PERIODIC) dy -= r.r.ny * rint(dy / r.r.ny);
        if (dims == 3 && r.bc_z == lbm::BC_PERIODIC) dz -= r.nz * rint(dz / r.nz);
        const double dist = sqrt(dx * dx + dy * dy + dz * dz);
        const double p = lbm::eval_pressure(r.r, rho);
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
        const double sp = sqrt(sp2);
        v[7] = sp == sp ? sp : INFINITY;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][tid] = v[q];
    __syncthreads();
    for (int s = kThreads3 / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int q = 0; q < 7; ++q) red[q][tid] += red[q][tid + s];
            red[7][tid] = fmax(red[7][tid], red[7][tid + s]);
        }
        __syncthreads();
    }
    if (tid < 8) partial[(int64_t)blockIdx.x * 8 + tid] = red[tid][0];
}

// ------------------------------------------------------------- launchers

static unsigned blocks3(int64_t n) { return (unsigned)((n + kThreads3 - 1) / kThreads3); }

template <typename S, int TX, int TY> hipError_t fused3_t(const Step3Args &a)
{
    const dim3 grid(fused3_blocks(a.nx, a.ny, a.nz, TX, TY, a.zchunk)), block(TX * TY);
    if (a.w32)
        hipExtLaunchKernelGGL((fused3_kernel<S, TX, TY, true>), grid, block, 0, a.stream, a.ev_col0, a.ev_col1, 0,
                              a.run, static_cast<const S *>(a.fin), static_cast<S *>(a.fout), a.status, a.zchunk);
    else
        hipExtLaunchKernelGGL((fused3_kernel<S, TX, TY, false>), grid, block, 0, a.stream, a.ev_col0, a.ev_col1, 0,
                              a.run, static_cast<const S *>(a.fin), static_cast<S *>(a.fout), a.status, a.zchunk);
    return hipGetLastError();
}

template <typename S> hipError_t fused3_shape(const Step3Args &a)
{
    switch (a.tile_x * 100 + a.tile_y) {
    case 3208: return fused3_t<S, 32, 8>(a);
    case 3216: return fused3_t<S, 32, 16>(a);
    case 6404: return fused3_t<S, 64, 4>(a);
    case 6416: return fused3_t<S, 64, 16>(a);
    default: return fused3_t<S, 64, 8>(a);
    }
}

template <typename S> hipError_t step3_t(const Step3Args &a)
{
    if (a.fused) return fused3_shape<S>(a);
    const unsigned nb = blocks3(a.nodes);
    hipExtLaunchKernelGGL(psi3_kernel<S>, dim3(nb), dim3(kThreads3), 0, a.stream, a.ev_psi0, a.ev_psi1, 0, a.run,
                          static_cast<const S *>(a.fin), a.psi, a.status);
    hipExtLaunchKernelGGL(collide3_kernel<S>, dim3(collide3_blocks(a.nx, a.ny, a.nz)), dim3(kThreads3), 0,
                          a.stream, a.ev_col0, a.ev_col1, 0, a.run, static_cast<const S *>(a.fin),
                          static_cast<S *>(a.fout), (const void *)a.psi, collide3_tile_shift(a.nx));
    return hipGetLastError();
}

hipError_t launch_step3(int precision, const Step3Args &a)
{
    return precision == PREC3_FP64 ? step3_t<double>(a) : step3_t<float>(a);
}

hipError_t launch_psi3(int precision, const Run3 *run, const void *f, void *psi, int32_t *status, int64_t nodes,
                       hipStream_t stream)
{
    if (precision == PREC3_FP64)
        psi3_kernel<double><<<blocks3(nodes), kThreads3, 0, stream>>>(run, static_cast<const double *>(f), psi, status);
    else
        psi3_kernel<float><<<blocks3(nodes), kThreads3, 0, stream>>>(run, static_cast<const float *>(f), psi, status);
    return hipGetLastError();
}

template <typename S>
hipError_t util3_t(int op, const Run3 *run, const void *fin, void *fout, const void *psi, double *buf, int64_t nodes,
                   hipStream_t stream)
{
    util3_kernel<S><<<blocks3(nodes), kThreads3, 0, stream>>>(run, op, static_cast<const S *>(fin),
                                                               static_cast<S *>(fout), psi, buf);
    return hipGetLastError();
}

hipError_t launch_util3(int precision, int op, const Run3 *run, const void *fin, void *fout, const void *psi,
                        double *buf, int64_t nodes, hipStream_t stream)
{
    return precision == PREC3_FP64 ? util3_t<double>(op, run, fin, fout, psi, buf, nodes, stream)
                                   : util3_t<float>(op, run, fin, fout, psi, buf, nodes, stream);
}

template <typename S>
hipError_t diag3_t(const Run3 *run, const void *f, const void *psi, int dims, double cx, double cy, double cz,
                   double r_in, double r_out, double *partial, int64_t nodes, hipStream_t stream)
{
    diag3_kernel<S><<<blocks3(nodes), kThreads3, 0, stream>>>(run, static_cast<const S *>(f), psi, dims, cx, cy, cz,
                                                               r_in, r_out, partial);
    return hipGetLastError();
}

hipError_t launch_diag3(int precision, const Run3 *run, const void *f, const void *psi, int dims, double cx,
                        double cy, double cz, double r_in, double r_out, double *partial, int64_t nodes,
                        hipStream_t stream)
{
    return precision == PREC3_FP64 ? diag3_t<double>(run, f, psi, dims, cx, cy, cz, r_in, r_out, partial, nodes, stream)
                                   : diag3_t<float>(run, f, psi, dims, cx, cy, cz, r_in, r_out, partial, nodes, stream);
}

} // namespace lbm3
