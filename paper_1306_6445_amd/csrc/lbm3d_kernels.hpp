// Launch interface of the D3Q19 kernels (lbm3d_kernels.hip), internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace lbm3 {

// D3Q19 velocities: rest, +-x, +-y, +-z, then the face diagonals in opposite pairs.
__host__ __device__ constexpr int ex3(int a)
{
    return a == 1 || a == 7 || a == 9 || a == 11 || a == 13 ? 1 : (a == 2 || a == 8 || a == 10 || a == 12 || a == 14 ? -1 : 0);
}
__host__ __device__ constexpr int ey3(int a)
{
    return a == 3 || a == 7 || a == 10 || a == 15 || a == 17 ? 1 : (a == 4 || a == 8 || a == 9 || a == 16 || a == 18 ? -1 : 0);
}
__host__ __device__ constexpr int ez3(int a)
{
    return a == 5 || a == 11 || a == 14 || a == 15 || a == 18 ? 1 : (a == 6 || a == 12 || a == 13 || a == 16 || a == 17 ? -1 : 0);
}
__host__ __device__ constexpr int opp3(int a) { return a == 0 ? 0 : (a % 2 ? a + 1 : a - 1); }

// Offsets of a node's two neighbours along one axis, in elements of a
// per-node array: to the node at c - 1 (m) and at c + 1 (p), wrapped on a
// periodic axis and 0 where a wall bounds the axis (psi beyond a wall is that
// of the adjacent fluid node, i.e. of the node itself along that axis); wm / wp
// tell whether a wall lies beyond that side (a population arriving from there
// is the node's own, reflected).
struct AxisNb {
    int64_t m, p;
    bool wm, wp;
};
__host__ __device__ inline AxisNb axis_nb(int c, int n, int bc, int64_t stride)
{
    AxisNb A;
    const bool wall = bc == lbm::BC_WALL;
    A.wm = wall && c == 0;
    A.wp = wall && c == n - 1;
    A.m = c > 0 ? -stride : (wall ? 0 : (int64_t)(n - 1) * stride);
    A.p = c < n - 1 ? stride : (wall ? 0 : -(int64_t)(n - 1) * stride);
    return A;
}
__host__ __device__ inline int64_t nb_off(const AxisNb &A, int e) { return e > 0 ? A.p : (e < 0 ? A.m : 0); }
__host__ __device__ inline bool nb_wall(const AxisNb &A, int e) { return e > 0 ? A.wp : (e < 0 && A.wm); }

// A population buffer holds the post-collision state: slot a of node y is
// f*_a(y).  The streamed population f_a(x) of node n (offsets X, Y, Z) is read
// from the upwind node's slot a, or from the node's own slot opp(a) where the
// upwind node lies beyond a wall (halfway bounce-back, Eq. 4); dstride
// elements separate one direction's slots from the next.  Every slot is the
// source of exactly one (node, direction) pair.
__host__ __device__ inline int64_t pull_slot3(int64_t n, const AxisNb &X, const AxisNb &Y, const AxisNb &Z, int a,
                                              int64_t dstride)
{
    const bool wall = nb_wall(X, -ex3(a)) || nb_wall(Y, -ey3(a)) || nb_wall(Z, -ez3(a));
    return wall ? (int64_t)opp3(a) * dstride + n
                : (int64_t)a * dstride + n + nb_off(X, -ex3(a)) + nb_off(Y, -ey3(a)) + nb_off(Z, -ez3(a));
}

// Node (x, y, z) of thread t in work item b of the collide pass (b after the
// XCD remap; tiles of 2^txs x (256 >> txs) nodes of one z-plane, x fastest,
// then y, then z); false for the threads of a ragged tile beyond the grid.
__host__ __device__ inline bool collide3_node(unsigned b, unsigned t, int nx, int ny, int nz, int txs, int &x, int &y,
                                              int &z)
{
    const int tys = 8 - txs; // 256 = 2^8 threads per workgroup
    const unsigned nbx = (unsigned)(nx + (1 << txs) - 1) >> txs, nby = (unsigned)(ny + (1 << tys) - 1) >> tys;
    const unsigned bxy = b % (nbx * nby);
    z = (int)(b / (nbx * nby));
    x = (int)((bxy % nbx) << txs) + (int)(t & ((1u << txs) - 1));
    y = (int)((bxy / nbx) << tys) + (int)(t >> txs);
    return x < nx && y < ny && z < nz;
}

// Indexing of one thread of the fused step (work item b after the XCD remap,
// thread t; tiles of TX x TY nodes, chunks of zc planes).  Its node (x, y) on
// planes [z0, z1) when active; the LDS cell of that node in a psi plane of
// (TX + 2) x (TY + 2) cells (the tile and a one-node ring) and the grid column
// (y * nx + x, wrapped or clamped: cx, cy) whose psi it computes there; when
// ring, also one ring cell and its column (rcx, rcy): rows -1 and TY of the
// tile, then columns -1 and TX.
struct Fused3Thread {
    int x, y, z0, z1, cell, rcell, cx, cy, rcx, rcy;
    bool active, ring;
    int64_t col, rcol;
};
__host__ __device__ inline Fused3Thread fused3_thread(unsigned b, int t, int nx, int ny, int nz, int bcx, int bcy,
                                                      int zc, int TX, int TY)
{
    Fused3Thread q;
    const int PX = TX + 2, RING = 2 * PX + 2 * TY;
    const unsigned ntx = (unsigned)(nx + TX - 1) / TX, nty = (unsigned)(ny + TY - 1) / TY;
    const unsigned bxy = b % (ntx * nty);
    q.z0 = (int)(b / (ntx * nty)) * zc;
    q.z1 = q.z0 + zc < nz ? q.z0 + zc : nz;
    const int x0 = (int)(bxy % ntx) * TX, y0 = (int)(bxy / ntx) * TY;
    const int lx = t % TX, ly = t / TX;
    q.x = x0 + lx;
    q.y = y0 + ly;
    q.active = q.x < nx && q.y < ny;
    q.cell = (ly + 1) * PX + lx + 1;
    q.cx = lbm::psi_coord(q.x, nx, bcx);
    q.cy = lbm::psi_coord(q.y, ny, bcy);
    q.col = (int64_t)q.cy * nx + q.cx;
    q.ring = t < RING;
    const int rx = t < 2 * PX ? t % PX - 1 : (t < 2 * PX + TY ? -1 : TX);
    const int ry = t < PX ? -1 : (t < 2 * PX ? TY : (t < 2 * PX + TY ? t - 2 * PX : t - 2 * PX - TY));
    q.rcell = (ry + 1) * PX + rx + 1;
    q.rcx = lbm::psi_coord(x0 + rx, nx, bcx);
    q.rcy = lbm::psi_coord(y0 + ry, ny, bcy);
    q.rcol = (int64_t)q.rcy * nx + q.rcx;
    return q;
}

// Per-run record of a 3D context in device memory.  The embedded 2D record
// carries the EOS, G, kappa and the FP32 base density in both arithmetic
// types (its nx, ny are the run's; pitch = nx).
struct alignas(16) Run3 {
    lbm::RunDev r;
    int32_t nz, bc_z, pad0[2];
    int64_t nodes;   // nx ny nz
    int64_t dstride; // elements from one direction's population array to the next
    double s[20];    // rates of the 19 moments (Lambda), padded
    float sf[20];
    double sig2;     // 2 sigma: the Eq. (8) flux shift is 2 sigma |F|^2 / psi^2 I
    float sig2f, pad1[3];
};

enum : int { PREC3_FP64 = 0, PREC3_FP32 = 1 };

struct Step3Args {
    const Run3 *run;
    const void *fin;
    void *fout;
    void *psi;
    int32_t *status;
    int64_t nodes;
    int32_t nx, ny, nz;
    int32_t fused = 1;   // 1: one fused launch per step; 0: psi pass + collide pass
    int32_t tile_x = 64; // fused: tile of tile_x x tile_y nodes, one thread each (fused3_shape_ok)
    int32_t tile_y = 8;
    int32_t zchunk = 64; // fused: planes one workgroup marches through
    bool w32 = false;    // each population buffer is below 4 GiB: 32-bit byte offsets in the fused kernel
    hipStream_t stream;
    hipEvent_t ev_psi0 = nullptr, ev_psi1 = nullptr, ev_col0 = nullptr, ev_col1 = nullptr;
};

// one time step fin -> fout: the fused launch, or the psi pass then the collide pass.
hipError_t launch_step3(int precision, const Step3Args &a);
// the psi pass alone (psi of the state f, for read-backs)
hipError_t launch_psi3(int precision, const Run3 *run, const void *f, void *psi, int32_t *status, int64_t nodes,
                       hipStream_t stream);
// FP64 host-order fields from the state fin: op 0 = populations [19][N] into
// buf, op 1 = density and Eq. (6) velocity [4][N] (needs psi of fin), op 2 =
// populations [19][N] from buf into fout (rounded to the storage), op 3 =
// equilibrium from buf (rho, ux, uy, uz [4][N]) into fout.
hipError_t launch_util3(int precision, int op, const Run3 *run, const void *fin, void *fout, const void *psi,
                        double *buf, int64_t nodes, hipStream_t stream);
// Per-block FP64 partial sums of the drop diagnostics (8 doubles per block:
// mass, sum rho_in, n_in, sum rho_out, n_out, sum p_in, sum p_out, max speed).
hipError_t launch_diag3(int precision, const Run3 *run, const void *f, const void *psi, int dims, double cx,
                        double cy, double cz, double r_in, double r_out, double *partial, int64_t nodes,
                        hipStream_t stream);
constexpr int kThreads3 = 256;
// collide pass: one workgroup per tile of 2^s x (256 >> s) nodes of one
// z-plane, 2^s the smallest power of two >= nx within [16, 256] (whole rows
// of up to 256 nodes per tile measured fastest; narrower grids stack rows)
inline int collide3_tile_shift(int64_t nx)
{
    int s = 4;
    while (s < 8 && ((int64_t)1 << s) < nx) ++s;
    return s;
}
// tile shapes of the fused step (threads per workgroup = tx ty)
inline bool fused3_shape_ok(int tx, int ty)
{
    return (tx == 32 && (ty == 8 || ty == 16)) || (tx == 64 && (ty == 4 || ty == 8 || ty == 16));
}
// workgroups of the fused step: x-y tiles of tx x ty nodes times chunks of zc planes
inline int64_t fused3_blocks(int64_t nx, int64_t ny, int64_t nz, int tx, int ty, int zc)
{
    return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + zc - 1) / zc);
}
// workgroups of the collide pass (a launch must stay below 2^32 threads:
// checked at validation)
inline int64_t collide3_blocks(int64_t nx, int64_t ny, int64_t nz)
{
    const int s = collide3_tile_shift(nx);
    const int64_t tx = (int64_t)1 << s, ty = kThreads3 >> s;
    return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * nz;
}

} // namespace lbm3
