// HIP kernels (gfx950) of the two-component (binary mixture) extension of the
// pseudopotential MRT step with the surface-tension source term (Li & Luo,
// arXiv:1306.6445, Section VI names multicomponent models as future work; the
// two-component form follows the derivation in the design notes).  One step
// is one launch of mc_fused_kernel:
//   each workgroup loads the populations of both components for its tile
//   (rows nodes per thread, ty rows apart) and a one-node ring around it,
//   sums the densities (psi_s = rho_s) into LDS, and after one barrier
//   collides every node of the tile: F_s (Eq. 7) and Q_s (Eq. 19) from the
//   other component's psi, the mixture velocity (Eq. 6 with both forces),
//   m_eq (Eq. 3) at rho_s and u, S (Eq. 5) with u and F_s, C (Eq. 18) with Q_s,
//   Eq. (17), f* = M^-1 m*, stored at the node in the second buffer.
// A buffer holds the post-collision state, streamed as it is read (Eq. 4;
// halfway bounce-back at walls: pull_slot2): loads are shifted by one node and
// stores aligned, which streams faster on this memory system than aligned
// loads with shifted stores.
#include <hip/hip_ext.h>

#include <type_traits>

#include "lbm3d_kernels.hpp"
#include "lbm_mc_kernels.hpp"

namespace lbmmc {

using lbm::ex_of;
using lbm::ey_of;
using lbm::opp_of;
using lbm3::AxisNb;
using lbm3::axis_nb;
using lbm3::nb_off;
using lbm3::nb_wall;

template <typename S> using ArithOf = typename std::conditional<std::is_same<S, double>::value, double, float>::type;

template <typename C> __device__ __forceinline__ C rate(const RunMC &r, int k)
{
    if constexpr (std::is_same<C, float>::value)
        return r.sf[k];
    else
        return r.s[k];
}

// FP32 storage: deviations f_a - w_a rho_ref[s] (the component's smallest
// initial density), decoded on load; FP64 stores the populations themselves.
template <typename C> __device__ __forceinline__ C ref_of(const RunMC &r, int s)
{
    if constexpr (std::is_same<C, float>::value)
        return r.rho_reff[s];
    else
        return C(0);
}
template <typename S, typename C> __device__ __forceinline__ C dec(S v, int a, C ref)
{
    if constexpr (std::is_same<S, double>::value)
        return v;
    else
        return v + C(lbm::rest_weight(a)) * ref;
}
template <typename S, typename C> __device__ __forceinline__ S enc(C v, int a, C ref)
{
    if constexpr (std::is_same<S, double>::value)
        return v;
    else
        return v - C(lbm::rest_weight(a)) * ref;
}

// f = M^-1 m for the orthogonal D2Q9 basis (the transform of the
// single-component kernels): M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6,
// 1/12, 1/4, 1/4), the conserved moments divided with the FMA-residual
// correction so that FP32 adds no mass or momentum bias.
template <typename C> __device__ __forceinline__ void mc_moments_to_pops(const C *m, C *f)
{
    const C a = lbm::div_const<C>(m[0], 9.0), b = m[1] * C(1.0 / 36.0), c = m[2] * C(1.0 / 36.0);
    const C d = lbm::div_const<C>(m[3], 6.0), e = m[4] * C(1.0 / 12.0), g = lbm::div_const<C>(m[5], 6.0);
    const C h = m[6] * C(1.0 / 12.0), i = m[7] * C(0.25), j = m[8] * C(0.25);
    const C ax = a - b - C(2) * c, dg = a + C(2) * b + c;
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

// Eq. (7) and Eq. (19) on component s from the other component's psi p[a] =
// psi_o(x + e_a) (p[0] at x) and its own psi_s.
template <typename C>
__device__ __forceinline__ void force_q(C G, C kappa, C psi_s, const C *p, C &Fx, C &Fy, C &Qxx, C &Qyy, C &Qxy)
{
    const C sx = C(1.0 / 3.0) * (p[1] - p[3]) + C(1.0 / 12.0) * ((p[5] - p[7]) + (p[8] - p[6]));
    const C sy = C(1.0 / 3.0) * (p[2] - p[4]) + C(1.0 / 12.0) * ((p[5] - p[7]) + (p[6] - p[8]));
    Fx = -G * psi_s * sx;
    Fy = -G * psi_s * sy;
    const C dsum = (p[5] + p[6]) + (p[7] + p[8]) - C(4) * p[0];
    const C kq = kappa * G * C(0.5) * psi_s;
    Qxx = kq * (C(1.0 / 3.0) * (p[1] + p[3] - C(2) * p[0]) + C(1.0 / 12.0) * dsum);
    Qyy = kq * (C(1.0 / 3.0) * (p[2] + p[4] - C(2) * p[0]) + C(1.0 / 12.0) * dsum);
    Qxy = kq * (C(1.0 / 12.0) * ((p[5] + p[7]) - (p[6] + p[8])));
}

// One component's collision at one node: its populations fv and density rs,
// the mixture velocity (ux, uy), its force and source tensor -> fs.
template <typename C>
__device__ __forceinline__ void collide_mc(const RunMC &r, const C *fv, C rs, C ux, C uy, C Fx, C Fy, C Qxx, C Qyy,
                                           C Qxy, C *fs)
{
    const C se = rate<C>(r, 1), sz = rate<C>(r, 2), sj = rate<C>(r, 3), sq = rate<C>(r, 4), sv = rate<C>(r, 7);
    const C sA = fv[1] + fv[3], sB = fv[2] + fv[4], sD = (fv[5] + fv[7]) + (fv[6] + fv[8]);
    const C d13 = fv[1] - fv[3], d24 = fv[2] - fv[4], d57 = fv[5] - fv[7], d86 = fv[8] - fv[6];
    const C jx = d13 + (d57 + d86), jy = d24 + (d57 - d86);
    const C sAB = sA + sB;
    const C m1 = C(-4) * fv[0] - sAB + C(2) * sD;
    const C m2 = C(4) * fv[0] - C(2) * sAB + sD;
    const C m4 = C(-2) * d13 + (d57 + d86), m6 = C(-2) * d24 + (d57 - d86);
    const C m7 = sA - sB, m8 = (fv[5] + fv[7]) - (fv[6] + fv[8]);
    // Eq. (3) at the component's density and the mixture velocity
    const C uxx = ux * ux, uyy = uy * uy, u2 = uxx + uyy;
    const C e1 = rs * (C(-2) + C(3) * u2), e2 = rs * (C(1) - C(3) * u2);
    const C e7 = rs * (uxx - uyy), e8 = rs * ux * uy;
    // Eq. (5) with the mixture velocity and the component's force
    const C S1 = C(6) * (ux * Fx + uy * Fy), S7 = C(2) * (ux * Fx - uy * Fy), S8 = ux * Fy + uy * Fx;
    // Eq. (18) with the component's Q
    const C trQ = Qxx + Qyy;
    const C C1 = C(1.5) * se * trQ, C2 = C(-1.5) * sz * trQ, C7 = -sv * (Qxx - Qyy), C8 = -sv * Qxy;
    // Eq. (17); the component's momentum relaxes toward rho_s u (inter-diffusion)
    C ms[9];
    ms[0] = rs;
    ms[1] = m1 - se * (m1 - e1) + (C(1) - C(0.5) * se) * S1 + C1;
    ms[2] = m2 - sz * (m2 - e2) - (C(1) - C(0.5) * sz) * S1 + C2;
    ms[3] = jx - sj * (jx - rs * ux) + (C(1) - C(0.5) * sj) * Fx;
    ms[4] = m4 - sq * (m4 + rs * ux) - (C(1) - C(0.5) * sq) * Fx;
    ms[5] = jy - sj * (jy - rs * uy) + (C(1) - C(0.5) * sj) * Fy;
    ms[6] = m6 - sq * (m6 + rs * uy) - (C(1) - C(0.5) * sq) * Fy;
    ms[7] = m7 - sv * (m7 - e7) + (C(1) - C(0.5) * sv) * S7 + C7;
    ms[8] = m8 - sv * (m8 - e8) + (C(1) - C(0.5) * sv) * S8 + C8;
    mc_moments_to_pops<C>(ms, fs);
}

// streamed populations of both components of node n (host-order index
// y nx + x, neighbour offsets X, Y)
template <typename S, typename C>
__device__ __forceinline__ void gather18(const S *__restrict__ f, int64_t N, int64_t n, const AxisNb &X,
                                         const AxisNb &Y, C refA, C refB, C *fa, C *fb)
{
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int64_t i = pull_slot2(n, X, Y, a, N);
        fa[a] = dec<S, C>(f[i], a, refA);
        fb[a] = dec<S, C>(f[9 * N + i], a, refB);
    }
}

// The same read for a buffer of less than 4 GiB: every slot's byte offset
// from the buffer's start fits in 32 bits, so each load takes one offset
// register beside the buffer's scalar base.  Offsets wrap modulo 2^32 and the
// final offset is exact.
template <typename S, typename C>
__device__ __forceinline__ void gather18_w32(const S *__restrict__ f, uint32_t N, uint32_t n, const AxisNb &X,
                                             const AxisNb &Y, C refA, C refB, C *fa, C *fb)
{
    const char *base = reinterpret_cast<const char *>(f);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const bool wall = nb_wall(X, -ex_of(a)) || nb_wall(Y, -ey_of(a));
        const uint32_t i = wall ? (uint32_t)opp_of(a) * N + n
                                : (uint32_t)a * N + n + (uint32_t)nb_off(X, -ex_of(a)) + (uint32_t)nb_off(Y, -ey_of(a));
        fa[a] = dec<S, C>(*reinterpret_cast<const S *>(base + (uint32_t)(i * (uint32_t)sizeof(S))), a, refA);
        fb[a] = dec<S, C>(*reinterpret_cast<const S *>(base + (uint32_t)((9 * N + i) * (uint32_t)sizeof(S))), a, refB);
    }
}

template <typename S, typename C, bool W32>
__device__ __forceinline__ void gather18_at(const S *__restrict__ f, int64_t N, int64_t n, const AxisNb &X,
                                            const AxisNb &Y, C refA, C refB, C *fa, C *fb)
{
    if constexpr (W32)
        gather18_w32<S, C>(f, (uint32_t)N, (uint32_t)n, X, Y, refA, refB, fa, fb);
    else
        gather18<S, C>(f, N, n, X, Y, refA, refB, fa, fb);
}

template <typename S, int R, bool W32>
__global__ void __launch_bounds__(512) mc_fused_kernel(const RunMC *__restrict__ runs, const S *__restrict__ fin,
                                                       S *__restrict__ fout, int32_t *__restrict__ status)
{
    using C = ArithOf<S>;
    extern __shared__ unsigned char lds_raw[];
    const RunMC &r = runs[0];
    const int nx = r.nx, ny = r.ny, bcx = r.bc_x, bcy = r.bc_y;
    const int TX = blockDim.x, TY = blockDim.y, TYR = R * TY, LX = TX + 2, LY = TYR + 2;
    C *la = reinterpret_cast<C *>(lds_raw);
    C *lb = la + LX * LY;
    int x0, y0;
    mc_tile_origin(lbm::work_index(1), nx, TX, TY, R, x0, y0);
    const int64_t N = r.dstride;
    const C refA = ref_of<C>(r, 0), refB = ref_of<C>(r, 1);
    bool bad = false;

    // the tile's own nodes (a column beyond the grid edge fills its LDS cell
    // with the wrapped or clamped node and collides nothing)
    const int x = x0 + (int)threadIdx.x;
    const int gx = lbm::psi_coord(x, nx, bcx);
    const AxisNb GX = axis_nb(gx, nx, bcx, 1);
    C fA[R][9], fB[R][9], rA[R], rB[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int y = y0 + (int)threadIdx.y + j * TY;
        const int gy = lbm::psi_coord(y, ny, bcy);
        gather18_at<S, C, W32>(fin, N, (int64_t)gy * nx + gx, GX, axis_nb(gy, ny, bcy, nx), refA, refB, fA[j], fB[j]);
        rA[j] = lbm::node_density<C>(fA[j]);
        rB[j] = lbm::node_density<C>(fB[j]);
        bad |= !(rA[j] + rB[j] > C(0)) || !(rA[j] - rA[j] == C(0)) || !(rB[j] - rB[j] == C(0));
        const int cell = ((int)threadIdx.y + j * TY + 1) * LX + (int)threadIdx.x + 1;
        la[cell] = rA[j];
        lb[cell] = rB[j];
    }
    // densities of the one-node ring: rows 0 and LY - 1 of the LDS tile, then columns 0 and LX - 1
    const int nring = 2 * LX + 2 * TYR;
    for (int k = (int)(threadIdx.y * TX + threadIdx.x); k < nring; k += TX * TY) {
        int lx, ly;
        mc_ring_cell(k, LX, LY, lx, ly);
        const int hx = lbm::psi_coord(x0 - 1 + lx, nx, bcx), hy = lbm::psi_coord(y0 - 1 + ly, ny, bcy);
        C ha[9], hb[9];
        gather18_at<S, C, W32>(fin, N, (int64_t)hy * nx + hx, axis_nb(hx, nx, bcx, 1), axis_nb(hy, ny, bcy, nx), refA,
                               refB, ha, hb);
        const C da = lbm::node_density<C>(ha), db = lbm::node_density<C>(hb);
        bad |= !(da + db > C(0)) || !(da - da == C(0)) || !(db - db == C(0));
        la[ly * LX + lx] = da;
        lb[ly * LX + lx] = db;
    }
    if (bad) status[0] = 1;
    __syncthreads();
    if (x >= nx) return;

    const C G = std::is_same<C, float>::value ? C(r.Gf) : C(r.G);
    const C kappa = std::is_same<C, float>::value ? C(r.kappaf) : C(r.kappa);
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int y = y0 + (int)threadIdx.y + j * TY;
        if (y >= ny) break;
        const int cell = ((int)threadIdx.y + j * TY + 1) * LX + (int)threadIdx.x + 1;
        C pA[9], pB[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            pA[a] = la[cell + ey_of(a) * LX + ex_of(a)];
            pB[a] = lb[cell + ey_of(a) * LX + ex_of(a)];
        }
        // psi_s = rho_s: A feels B's psi and B feels A's
        C FAx, FAy, QAxx, QAyy, QAxy, FBx, FBy, QBxx, QByy, QBxy;
        force_q<C>(G, kappa, rA[j], pB, FAx, FAy, QAxx, QAyy, QAxy);
        force_q<C>(G, kappa, rB[j], pA, FBx, FBy, QBxx, QByy, QBxy);
        // Eq. (6) for the mixture
        C jx = C(0), jy = C(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const C v = fA[j][a] + fB[j][a];
            if (ex_of(a)) jx += C(ex_of(a)) * v;
            if (ey_of(a)) jy += C(ey_of(a)) * v;
        }
        const C irho = lbm::recip<C>(rA[j] + rB[j]);
        const C ux = (jx + C(0.5) * (FAx + FBx)) * irho, uy = (jy + C(0.5) * (FAy + FBy)) * irho;
        C sa[9], sb[9];
        collide_mc<C>(r, fA[j], rA[j], ux, uy, FAx, FAy, QAxx, QAyy, QAxy, sa);
        collide_mc<C>(r, fB[j], rB[j], ux, uy, FBx, FBy, QBxx, QByy, QBxy, sb);
        // f* stays at the node; the next read streams it (Eq. 4)
        const int64_t n = (int64_t)y * nx + x;
        if constexpr (W32) {
            char *base = reinterpret_cast<char *>(fout);
            const uint32_t N32 = (uint32_t)N, n32 = (uint32_t)n;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                *reinterpret_cast<S *>(base + (uint32_t)(((uint32_t)a * N32 + n32) * (uint32_t)sizeof(S))) =
                    enc<S, C>(sa[a], a, refA);
                *reinterpret_cast<S *>(base + (uint32_t)(((uint32_t)(9 + a) * N32 + n32) * (uint32_t)sizeof(S))) =
                    enc<S, C>(sb[a], a, refB);
            }
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                fout[(int64_t)a * N + n] = enc<S, C>(sa[a], a, refA);
                fout[(int64_t)(9 + a) * N + n] = enc<S, C>(sb[a], a, refB);
            }
        }
    }
}

// ------------------------------------------------------------- utilities

template <typename S>
__global__ void __launch_bounds__(kThreadsMC) util_mc_kernel(const RunMC *__restrict__ runs, int op,
                                                             const S *__restrict__ fin, S *__restrict__ fout,
                                                             double *__restrict__ buf)
{
    using C = ArithOf<S>;
    const RunMC &r = runs[0];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t NN = r.nodes, N = r.dstride;
    if (n >= NN) return;
    const C ref[2] = {ref_of<C>(r, 0), ref_of<C>(r, 1)};
    const int x = (int)(n % r.nx), y = (int)(n / r.nx);
    const AxisNb X = axis_nb(x, r.nx, r.bc_x, 1), Y = axis_nb(y, r.ny, r.bc_y, r.nx);
    // slot of the streamed population f_a(x) of component s (reads), and
    // where a state given as f_a(x) goes (writes: each slot once)
    auto slot = [&](int s, int a) { return (int64_t)s * 9 * N + pull_slot2(n, X, Y, a, N); };
    if (op == 0) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 9; ++a)
                buf[(int64_t)(s * 9 + a) * NN + n] = (double)dec<S, C>(fin[slot(s, a)], a, ref[s]);
    } else if (op == 1) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 9; ++a) fout[slot(s, a)] = enc<S, C>((C)buf[(int64_t)(s * 9 + a) * NN + n], a, ref[s]);
    } else if (op == 2) {
        // f = M^-1 m_eq(rho_s, u) (Eq. 3), in FP64 then rounded to the storage
        const double ux = buf[2 * NN + n], uy = buf[3 * NN + n], u2 = ux * ux + uy * uy;
        for (int s = 0; s < 2; ++s) {
            const double rho = buf[s * NN + n];
            const double m[9] = {rho, rho * (-2.0 + 3.0 * u2), rho * (1.0 - 3.0 * u2), rho * ux, -rho * ux,
                                 rho * uy, -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy};
            double fd[9];
            mc_moments_to_pops<double>(m, fd);
#pragma unroll
            for (int a = 0; a < 9; ++a) fout[slot(s, a)] = enc<S, C>((C)fd[a], a, ref[s]);
        }
    } else if (op == 3) {
        for (int s = 0; s < 2; ++s) {
            double rho = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) rho += (double)dec<S, C>(fin[slot(s, a)], a, ref[s]);
            buf[s * NN + n] = rho;
        }
    } else {
        // Eq. (6) for the mixture, FP64, from the densities in buf[0, 2N)
        double pA[9], pB[9];
        for (int a = 0; a < 9; ++a) {
            const int64_t m = (int64_t)lbm::psi_coord(y + ey_of(a), r.ny, r.bc_y) * r.nx +
                              lbm::psi_coord(x + ex_of(a), r.nx, r.bc_x);
            pA[a] = buf[m];
            pB[a] = buf[NN + m];
        }
        double FAx, FAy, FBx, FBy, q0, q1, q2;
        force_q<double>(r.G, 0.0, pA[0], pB, FAx, FAy, q0, q1, q2);
        force_q<double>(r.G, 0.0, pB[0], pA, FBx, FBy, q0, q1, q2);
        double jx = 0.0, jy = 0.0;
        for (int s = 0; s < 2; ++s)
            for (int a = 1; a < 9; ++a) {
                const double v = (double)dec<S, C>(fin[slot(s, a)], a, ref[s]);
                jx += ex_of(a) * v;
                jy += ey_of(a) * v;
            }
        const double rho = pA[0] + pB[0];
        buf[2 * NN + n] = (jx + 0.5 * (FAx + FBx)) / rho;
        buf[3 * NN + n] = (jy + 0.5 * (FAy + FBy)) / rho;
    }
}

__global__ void __launch_bounds__(kThreadsMC) diag_mc_kernel(const RunMC *__restrict__ runs,
                                                             const double *__restrict__ buf, double cx, double cy,
                                                             double r_in, double r_out, double *__restrict__ partial)
{
    __shared__ double red[kDiagMC][kThreadsMC];
    const RunMC &r = runs[0];
    const int64_t NN = r.nodes, n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int tid = threadIdx.x;
    double v[kDiagMC] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (n < NN) {
        const double a = buf[n], b = buf[NN + n], ux = buf[2 * NN + n], uy = buf[3 * NN + n];
        const int x = (int)(n % r.nx), y = (int)(n / r.nx);
        double dx = x - cx, dy = y - cy;
        if (r.bc_x == lbm::BC_PERIODIC) dx -= r.nx * rint(dx / r.nx);
        if (r.bc_y == lbm::BC_PERIODIC) dy -= r.ny * rint(dy / r.ny);
        const double dist = sqrt(dx * dx + dy * dy);
        // bulk pressure of the mixture: (rho_A + rho_B) / 3 + G rho_A rho_B
        const double p = (a + b) / 3.0 + r.G * a * b;
        v[0] = a;
        v[1] = b;
        if (dist <= r_in) {
            v[2] = a;
            v[3] = b;
            v[4] = 1.0;
            v[8] = p;
        }
        if (dist >= r_out) {
            v[5] = a;
            v[6] = b;
            v[7] = 1.0;
            v[9] = p;
        }
        const double sp = sqrt(ux * ux + uy * uy);
        v[10] = sp == sp ? sp : INFINITY;
    }
#pragma unroll
    for (int q = 0; q < kDiagMC; ++q) red[q][tid] = v[q];
    __syncthreads();
    for (int s = kThreadsMC / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int q = 0; q < kDiagMC - 1; ++q) red[q][tid] += red[q][tid + s];
            red[kDiagMC - 1][tid] = fmax(red[kDiagMC - 1][tid], red[kDiagMC - 1][tid + s]);
        }
        __syncthreads();
    }
    if (tid < kDiagMC) partial[(int64_t)blockIdx.x * kDiagMC + tid] = red[tid][0];
}

// ------------------------------------------------------------- launchers

template <typename S, int R> hipError_t fused_mc_t(const StepMCArgs &a)
{
    using C = ArithOf<S>;
    const uint32_t lds = 2 * sizeof(C) * (a.tx + 2) * (R * a.ty + 2);
    const int64_t tiles = mc_tiles(a.nx, a.ny, a.tx, a.ty, R);
    if (a.w32)
        hipExtLaunchKernelGGL((mc_fused_kernel<S, R, true>), dim3((unsigned)tiles), dim3(a.tx, a.ty), lds, a.stream,
                              a.ev0, a.ev1, 0, a.run, static_cast<const S *>(a.fin), static_cast<S *>(a.fout), a.status);
    else
        hipExtLaunchKernelGGL((mc_fused_kernel<S, R, false>), dim3((unsigned)tiles), dim3(a.tx, a.ty), lds, a.stream,
                              a.ev0, a.ev1, 0, a.run, static_cast<const S *>(a.fin), static_cast<S *>(a.fout), a.status);
    return hipGetLastError();
}

template <typename S> hipError_t step_mc_t(const StepMCArgs &a)
{
    switch (a.rows) {
    case 1: return fused_mc_t<S, 1>(a);
    case 4: return fused_mc_t<S, 4>(a);
    default: return fused_mc_t<S, 2>(a);
    }
}

hipError_t launch_step_mc(int precision, const StepMCArgs &a)
{
    if (!mc_shape_ok(a.tx, a.ty, a.rows)) return hipErrorInvalidValue;
    return precision == PRECMC_FP64 ? step_mc_t<double>(a) : step_mc_t<float>(a);
}

static unsigned blocks_mc(int64_t n) { return (unsigned)((n + kThreadsMC - 1) / kThreadsMC); }

hipError_t launch_util_mc(int precision, int op, const RunMC *run, const void *fin, void *fout, double *buf,
                          int64_t nodes, hipStream_t stream)
{
    if (precision == PRECMC_FP64)
        util_mc_kernel<double><<<blocks_mc(nodes), kThreadsMC, 0, stream>>>(run, op, static_cast<const double *>(fin),
                                                                             static_cast<double *>(fout), buf);
    else
        util_mc_kernel<float><<<blocks_mc(nodes), kThreadsMC, 0, stream>>>(run, op, static_cast<const float *>(fin),
                                                                            static_cast<float *>(fout), buf);
    return hipGetLastError();
}

hipError_t launch_diag_mc(const RunMC *run, const double *buf, double cx, double cy, double r_in, double r_out,
                          double *partial, int64_t nodes, hipStream_t stream)
{
    diag_mc_kernel<<<blocks_mc(nodes), kThreadsMC, 0, stream>>>(run, buf, cx, cy, r_in, r_out, partial);
    return hipGetLastError();
}

} // namespace lbmmc
