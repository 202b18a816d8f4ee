// Device-side building blocks of the MI355X lattice Boltzmann path: the
// per-run descriptor, the pseudopotential / EOS evaluation (Section II,
// Eq. 23), population storage codecs and the in-place AA addressing of
// streaming (Eq. 4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

// D2Q9 velocities, e0..e8 as in Section II.
__host__ __device__ constexpr int ex_of(int a) { return a == 1 || a == 5 || a == 8 ? 1 : (a == 3 || a == 6 || a == 7 ? -1 : 0); }
__host__ __device__ constexpr int ey_of(int a) { return a == 2 || a == 5 || a == 6 ? 1 : (a == 4 || a == 7 || a == 8 ? -1 : 0); }
__host__ __device__ constexpr int opp_of(int a) { return a == 0 ? 0 : (a <= 4 ? ((a + 1) & 3) + 1 : ((a - 3) & 3) + 5); }

// Lattice weights of the rest state (used by the deviation storage codecs).
__host__ __device__ constexpr double rest_weight(int a) { return a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

enum : int { EOS_CS = 0, EOS_PIECEWISE = 1, EOS_EXP = 2 };
enum : int { BC_PERIODIC = 0, BC_WALL = 1 };

// Per-run constants in one arithmetic type: the FP64 kernels read the
// double set, the FP32 and bf16-storage kernels the float set (the host
// rounds each constant once), so no double arithmetic runs in their step.
template <typename C> struct RunPar {
    C eos[6];     // EOS parameters as in lbm.h (CS: a, b, R, T ...)
    C G;
    C kappa;
    C sig_coef;   // 12 sigma / (tau_e - 1/2), Eq. (8) with dt = 1
    C s_e, s_zeta, s_q, s_nu;
    C rho_ref;    // base density of the FP32 deviation storage (bf16: per population, see Store)
    C rho_nu;     // step-function viscosity (Section V.C): below rho_nu the stress
    C s_nu_low;   // moments relax at s_nu_low instead of s_nu (rho_nu = 0: off)
    C G2;         // multi-range potential, Eq. (9): G acts on x + e_a, G2 on x + 2 e_a
    C G_eos;      // G1 + 2 G2: the interaction strength of the EOS (Section III.A)
    C eta_scale;  // Carnahan-Starling: eta = (b / 4) rho
    C RT;         // Carnahan-Starling: R T
    C two_over_G; // 2 / G_eos (the sqrt pseudopotential's radicand factor)
    C pad;
};

// Per-run record in device memory.
struct alignas(16) RunDev {
    int32_t nx, ny, bc_x, bc_y;
    int64_t f_off;   // element offset of the run's population block [9][dstride]
    int64_t n_off;   // element offset of the run's node arrays [ny][pitch]
    int64_t dstride; // elements from one direction's array to the next (>= pitch * ny)
    int32_t eos_kind, tile_begin, tile_count; // tile_begin / tile_count: the run's range of the work list
    int32_t pitch;   // row stride of the run's device arrays (>= nx; the host sets nx)
    int32_t pad0[2];
    RunPar<double> pd;
    RunPar<float> pf;
    int32_t pad1[2];

    template <typename C> __host__ __device__ __forceinline__ const RunPar<C> &par() const;
};
template <> __host__ __device__ __forceinline__ const RunPar<double> &RunDev::par<double>() const { return pd; }
template <> __host__ __device__ __forceinline__ const RunPar<float> &RunDev::par<float>() const { return pf; }
static_assert(sizeof(RunPar<double>) == 176 && sizeof(RunPar<float>) == 88, "RunPar layout");
static_assert(sizeof(RunDev) == 336, "RunDev layout");

// Fills the derived constants of pd and the rounded float set from the
// primary fields of pd (host side, before every upload of the record).
inline void finish_rundev(RunDev &r)
{
    RunPar<double> &d = r.pd;
    d.eta_scale = d.eos[1] * 0.25;
    d.RT = d.eos[2] * d.eos[3];
    d.two_over_G = d.G_eos != 0.0 ? 2.0 / d.G_eos : 0.0;
    d.pad = 0.0;
    const double *src = &d.eos[0];
    float *dst = &r.pf.eos[0];
    for (int i = 0; i < (int)(sizeof(RunPar<double>) / sizeof(double)); ++i) dst[i] = (float)src[i];
}

// Tile of the work list: run id and the tile's origin in that run.
struct alignas(16) Tile {
    int32_t run, x0, y0, pad;
};

// ------------------------------------------------------------ bf16 codec
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ uint16_t float_to_bf16_rne(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u); // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Stochastic rounding: r16 uniform in [0, 2^16) added below the 16 kept bits,
// then truncation, rounds the magnitude up with probability equal to the
// discarded fraction, so the rounding error has zero mean.
__device__ __forceinline__ uint16_t float_to_bf16_sr(float v, uint32_t r16)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return (uint16_t)((u + r16) >> 16);
}

// MurmurHash3's 32-bit finalizer (fmix32, A. Appleby): a bijective avalanche
// mix, used as a counter-based source of rounding bits.
__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Storage traits: S is what lives in HBM, C is the arithmetic type.
template <typename S> struct Store;

template <> struct Store<double> {
    using C = double;
    template <int A> __device__ static __forceinline__ double load(const double *p, int64_t i, double) { return p[i]; }
    template <int A> __device__ static __forceinline__ void store(double *p, int64_t i, double v, double) { p[i] = v; }
};

// FP32 and bf16 storage keep deviations f_a - w_a rho_ref from the rest state
// at a per-run base density: the stored numbers are small where the density is
// near rho_ref, and so is their rounding.
template <> struct Store<float> {
    using C = float;
    template <int A> __device__ static __forceinline__ float load(const float *p, int64_t i, float ref)
    {
        return p[i] + (float)rest_weight(A) * ref;
    }
    template <int A> __device__ static __forceinline__ void store(float *p, int64_t i, float v, float ref)
    {
        p[i] = v - (float)rest_weight(A) * ref;
    }
};

// bf16 storage takes its base density per population: the density that the
// node which wrote the population had when it wrote it (see upwind_node), so
// that the stored number is only the non-rest part w_a rho (3 e.v + ...) plus
// the non-equilibrium part, in liquid and vapour alike.
template <> struct Store<bf16_t> {
    using C = float;
    template <int A> __device__ static __forceinline__ float load(const bf16_t *p, int64_t i, float ref)
    {
        return bf16_to_float(p[i].bits) + (float)rest_weight(A) * ref;
    }
    template <int A> __device__ static __forceinline__ void store(bf16_t *p, int64_t i, float v, float ref)
    {
        p[i].bits = float_to_bf16_rne(v - (float)rest_weight(A) * ref);
    }
    template <int A>
    __device__ static __forceinline__ void store_sr(bf16_t *p, int64_t i, float v, float ref, uint32_t r16)
    {
        p[i].bits = float_to_bf16_sr(v - (float)rest_weight(A) * ref, r16);
    }
};

// Storage whose base density is the writer's density (one FP32 density array
// per step parity) rather than a per-run constant.
template <typename S> constexpr bool kWriterRef = std::is_same<S, bf16_t>::value;

// ------------------------------------------------------------ divisions
// FP32: 1/x as the hardware reciprocal refined by one Newton step; x/d for a
// small constant d as the product with the rounded reciprocal, corrected once
// by its exact FMA residual (within an ulp of the quotient, without bias).
// Each replaces a division sequence of about ten instructions in kernels
// that are partly issue-bound.  FP64 keeps the IEEE division.
template <typename C> __device__ __forceinline__ C recip(C x)
{
    if constexpr (std::is_same<C, float>::value) {
        const float r = __builtin_amdgcn_rcpf(x);
        return fmaf(r, fmaf(-x, r, 1.0f), r);
    } else {
        return C(1) / x;
    }
}
template <typename C> __device__ __forceinline__ C div_const(C x, double d)
{
    if constexpr (std::is_same<C, float>::value) {
        const float inv = (float)(1.0 / d), q = x * inv;
        return fmaf(fmaf(-q, (float)d, x), inv, q);
    } else {
        return x / C(d);
    }
}

// ------------------------------------------------------------------ EOS
// psi(rho) of the three pseudopotential forms; returns false where psi is not
// real (rho <= 0, eta >= 1, or p_EOS > rho / 3 with G < 0).
template <typename C>
__device__ __forceinline__ bool eval_psi(const RunDev &r, C rho, C &psi)
{
    const RunPar<C> &k = r.template par<C>();
    if (!(rho > C(0))) return false;
    if (r.eos_kind == EOS_EXP) {
        psi = k.eos[0] * exp(-k.eos[1] / rho);
        return true;
    }
    C p;
    if (r.eos_kind == EOS_CS) {
        const C a = k.eos[0], RT = k.RT;
        const C eta = k.eta_scale * rho;
        if (!(eta < C(1))) return false;
        const C om = C(1) - eta;
        p = rho * RT * (C(1) + eta * (C(1) + eta * (C(1) - eta))) * recip<C>(om * om * om) - a * rho * rho;
    } else {
        const C thV = k.eos[0], thM = k.eos[1], thL = k.eos[2];
        const C r1 = k.eos[3], r2 = k.eos[4];
        if (rho <= r1)
            p = rho * thV;
        else if (rho < r2)
            p = r1 * thV + (rho - r1) * thM;
        else
            p = r1 * thV + (r2 - r1) * thM + (rho - r2) * thL;
    }
    C rad;
    if constexpr (std::is_same<C, float>::value)
        rad = (p - rho * C(1.0 / 3.0)) * k.two_over_G;
    else
        rad = C(2) * (p - rho * C(1.0 / 3.0)) / k.G_eos;
    if (!(rad >= C(0))) return false;
    psi = sqrt(rad);
    return true;
}

// Bulk pressure p_EOS(rho) in FP64 (diagnostics only).
__device__ __forceinline__ double eval_pressure(const RunDev &r, double rho)
{
    const RunPar<double> &k = r.pd;
    if (r.eos_kind == EOS_EXP) {
        const double psi = k.eos[0] * exp(-k.eos[1] / rho);
        return rho / 3.0 + k.G_eos * psi * psi * 0.5;
    }
    if (r.eos_kind == EOS_CS) {
        const double eta = k.eos[1] * 0.25 * rho, om = 1.0 - eta;
        return rho * k.eos[2] * k.eos[3] * (1.0 + eta * (1.0 + eta * (1.0 - eta))) / (om * om * om) -
               k.eos[0] * rho * rho;
    }
    const double thV = k.eos[0], thM = k.eos[1], thL = k.eos[2], r1 = k.eos[3], r2 = k.eos[4];
    if (rho <= r1) return rho * thV;
    if (rho < r2) return r1 * thV + (rho - r1) * thM;
    return r1 * thV + (r2 - r1) * thM + (rho - r2) * thL;
}

// Eq. (6) density of one node from its nine populations.  FP64: a pairwise
// sum in a fixed order.  FP32: the same tree with every addition made
// error-free by Knuth's TwoSum (s + e = a + b exactly, six additions, no
// ordering condition), the error terms summed and added once, so the density
// is the exact sum rounded about once and carries no systematic rounding bias
// (a plain FP32 sum of nine populations is off by a few ulps, the same way at
// every node of a uniform phase).
__device__ __forceinline__ float two_sum(float a, float b, float &e)
{
    const float s = a + b;
    const float bv = s - a;
    e = (a - (s - bv)) + (b - bv);
    return s;
}

template <typename C> __device__ __forceinline__ C node_density(const C *f)
{
    if constexpr (std::is_same<C, float>::value) {
        float e13, e24, e57, e68, e0, e1, e2, e3;
        const float s13 = two_sum(f[1], f[3], e13), s24 = two_sum(f[2], f[4], e24);
        const float s57 = two_sum(f[5], f[7], e57), s68 = two_sum(f[6], f[8], e68);
        const float a = two_sum(f[0], s13, e0);
        const float b = two_sum(a, s24, e1);
        const float d = two_sum(s57, s68, e2);
        const float s = two_sum(b, d, e3);
        return s + (((e13 + e24) + (e57 + e68)) + ((e0 + e1) + (e2 + e3)));
    } else {
        return ((f[0] + (f[1] + f[3])) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8]));
    }
}

// --------------------------------------------------------- AA addressing
// State at an even step count: slot a of node x holds f_a(x).
// State at an odd step count: f_a(x) sits in slot opp(a) of node x - e_a, or,
// when x - e_a lies beyond a wall, in slot a of x itself (halfway bounce-back).
// An even step reads and writes only its own node (writes go to opposite
// slots); an odd step reads where the odd-state rule says and writes f*_a to
// slot a of x + e_a (or to slot opp(a) of x across a wall).  Each node touches
// the same nine addresses for reading and writing, so the update is in place.
struct Nbr {
    int32_t xm, xp, ym, yp; // wrapped neighbour coordinates
    bool wxm, wxp, wym, wyp; // neighbour lies beyond a wall
};

__host__ __device__ __forceinline__ Nbr neighbours(int x, int y, int nx, int ny, int bcx, int bcy)
{
    Nbr n;
    n.xm = x == 0 ? nx - 1 : x - 1;
    n.xp = x == nx - 1 ? 0 : x + 1;
    n.ym = y == 0 ? ny - 1 : y - 1;
    n.yp = y == ny - 1 ? 0 : y + 1;
    n.wxm = bcx == BC_WALL && x == 0;
    n.wxp = bcx == BC_WALL && x == nx - 1;
    n.wym = bcy == BC_WALL && y == 0;
    n.wyp = bcy == BC_WALL && y == ny - 1;
    return n;
}

// Flat index (within a run's block) of the slot holding f_a(x) in the odd
// state, i.e. where the odd step reads direction a and writes direction opp(a).
// ld: row stride of the block, N: stride between directions.
template <int A>
__host__ __device__ __forceinline__ int64_t odd_slot(int x, int y, const Nbr &n, int ld, int64_t N)
{
    constexpr int ex = ex_of(A), ey = ey_of(A);
    const bool wall = (ex > 0 && n.wxm) || (ex < 0 && n.wxp) || (ey > 0 && n.wym) || (ey < 0 && n.wyp);
    if (wall) return (int64_t)A * N + (int64_t)y * ld + x;
    const int sx = ex > 0 ? n.xm : (ex < 0 ? n.xp : x);
    const int sy = ey > 0 ? n.ym : (ey < 0 ? n.yp : y);
    return (int64_t)opp_of(A) * N + (int64_t)sy * ld + sx;
}

template <int A>
__host__ __device__ __forceinline__ int64_t even_slot(int x, int y, int ld, int64_t N)
{
    return (int64_t)A * N + (int64_t)y * ld + x;
}

// The odd-state slot of f_a(x) for a node whose neighbours lie inside the
// grid, not across a periodic seam or a wall: slot opp(a) of x - e_a, a fixed
// offset from the node's flat index idx (within the run).
template <int A>
__host__ __device__ __forceinline__ int64_t odd_slot_inner(int64_t idx, int ld, int64_t N)
{
    return (int64_t)opp_of(A) * N + idx - (ey_of(A) * ld + ex_of(A));
}

// Node that wrote f_a(x) during the previous step (Eq. 4: f_a(x, t+1) =
// f*_a(x - e_a, t)): x - e_a, or x itself when x - e_a lies beyond a wall
// (halfway bounce-back returns the population to the node that sent it).
// Flat index within the run (row stride ld).  The same node holds the
// odd-state slot.
template <int A>
__host__ __device__ __forceinline__ int64_t upwind_node(int x, int y, const Nbr &n, int ld)
{
    constexpr int ex = ex_of(A), ey = ey_of(A);
    const bool wall = (ex > 0 && n.wxm) || (ex < 0 && n.wxp) || (ey > 0 && n.wym) || (ey < 0 && n.wyp);
    if (wall) return (int64_t)y * ld + x;
    const int sx = ex > 0 ? n.xm : (ex < 0 ? n.xp : x);
    const int sy = ey > 0 ? n.ym : (ey < 0 ? n.yp : y);
    return (int64_t)sy * ld + sx;
}

// The same node as an offset in an LDS tile with row stride LX centred on x.
template <int A>
__host__ __device__ __forceinline__ int upwind_offset(const Nbr &n, int LX)
{
    constexpr int ex = ex_of(A), ey = ey_of(A);
    const bool wall = (ex > 0 && n.wxm) || (ex < 0 && n.wxp) || (ey > 0 && n.wym) || (ey < 0 && n.wyp);
    return wall ? 0 : -ey * LX - ex;
}

__host__ __device__ __forceinline__ int64_t upwind_node_rt(int a, int x, int y, const Nbr &n, int ld)
{
    const int ex = ex_of(a), ey = ey_of(a);
    const bool wall = (ex > 0 && n.wxm) || (ex < 0 && n.wxp) || (ey > 0 && n.wym) || (ey < 0 && n.wyp);
    if (wall) return (int64_t)y * ld + x;
    const int sx = ex > 0 ? n.xm : (ex < 0 ? n.xp : x);
    const int sy = ey > 0 ? n.ym : (ey < 0 ? n.yp : y);
    return (int64_t)sy * ld + sx;
}

// Coordinate of a psi neighbour: periodic wrap, or clamp across a wall.
__host__ __device__ __forceinline__ int psi_coord(int c, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        // one wrap covers a halo narrower than the grid; the remainder only
        // for grids narrower than their halo
        c = c < 0 ? c + n : (c >= n ? c - n : c);
        if (c < 0 || c >= n) {
            c %= n;
            if (c < 0) c += n;
        }
        return c;
    }
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// Work-list index of this workgroup.  Workgroups are dispatched to the eight
// XCDs round-robin (block b runs on XCD b % 8); with `xcd` set, XCD k walks a
// contiguous range of the work list, so tiles that share halo rows and edge
// cache lines run under the same L2.
constexpr int kNumXcd = 8;

__host__ __device__ __forceinline__ int work_index_of(int b, int n, int xcd)
{
    if (!xcd) return b;
    const int q = n / kNumXcd, r = n % kNumXcd;
    const int k = b % kNumXcd;
    return k * q + (k < r ? k : r) + b / kNumXcd;
}

__device__ __forceinline__ int work_index(int xcd) { return work_index_of(blockIdx.x, gridDim.x, xcd); }

template <int A, typename F> struct Unroll {
    __device__ __forceinline__ static void run(F &f)
    {
        Unroll<A - 1, F>::run(f);
        f.template operator()<A - 1>();
    }
};
template <typename F> struct Unroll<0, F> {
    __device__ __forceinline__ static void run(F &) {}
};
template <typename F> __device__ __forceinline__ void for9(F &f) { Unroll<9, F>::run(f); }

} // namespace lbm
