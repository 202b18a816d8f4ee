// Launch interface of the two-component (binary mixture) kernels
// (lbm_mc_kernels.hip), internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm3d_kernels.hpp"
#include "lbm_device.hpp"

namespace lbmmc {

// Per-run record of a two-component context in device memory.  Populations
// f[s][a][y][x]: component s = 0 (A) or 1 (B), direction a; one direction's
// array is dstride elements, one component's 9 dstride.
struct alignas(16) RunMC {
    int32_t nx, ny, bc_x, bc_y;
    int64_t nodes;
    int64_t dstride;
    double G, kappa;     // cross interaction (> 0), Eq. (19)
    double s[9];         // Lambda in moment order
    double rho_ref[2];   // FP32 storage: f_a - w_a rho_ref[s] per component
    float Gf, kappaf;
    float sf[9];
    float rho_reff[2];
    float pad[3];
};

enum : int { PRECMC_FP64 = 0, PRECMC_FP32 = 1 };

// One fused step (fin -> fout) over tiles of tx x (rows ty) nodes.
struct StepMCArgs {
    const RunMC *run;
    const void *fin;
    void *fout;
    int32_t *status;
    int32_t nx, ny;
    int32_t tx = 128, ty = 4, rows = 1; // threads per tile (tx x ty), nodes per thread (rows, ty apart)
    bool w32 = false;                    // each population buffer is below 4 GiB: 32-bit byte offsets
    hipStream_t stream;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// A population buffer holds the post-collision state: slot (s, a) of node y
// is f*_a(y) of component s.  The streamed population f_a(x) of node n (x and
// y neighbour offsets X, Y as in the 3D extension) is read from the upwind
// node's slot a, or from the node's own slot opp(a) where the upwind node lies
// beyond a wall (halfway bounce-back, Eq. 4); component B's slots follow
// component A's 9 N elements later.  Every slot is the source of exactly one
// (node, direction) pair.
__host__ __device__ inline int64_t pull_slot2(int64_t n, const lbm3::AxisNb &X, const lbm3::AxisNb &Y, int a,
                                              int64_t N)
{
    const int ex = lbm::ex_of(a), ey = lbm::ey_of(a);
    const bool wall = lbm3::nb_wall(X, -ex) || lbm3::nb_wall(Y, -ey);
    return wall ? (int64_t)lbm::opp_of(a) * N + n : (int64_t)a * N + n + lbm3::nb_off(X, -ex) + lbm3::nb_off(Y, -ey);
}

// tile shapes: tx in {32, 64, 128, 256}, ty in {1, 2, 4, 8}, 64 <= tx ty <= 512, rows in {1, 2, 4}
inline bool mc_shape_ok(int tx, int ty, int rows)
{
    const bool okx = tx == 32 || tx == 64 || tx == 128 || tx == 256;
    const bool oky = ty == 1 || ty == 2 || ty == 4 || ty == 8;
    return okx && oky && tx * ty >= 64 && tx * ty <= 512 && (rows == 1 || rows == 2 || rows == 4);
}
inline int64_t mc_tiles(int64_t nx, int64_t ny, int tx, int ty, int rows)
{
    const int64_t th = (int64_t)ty * rows;
    return ((nx + tx - 1) / tx) * ((ny + th - 1) / th);
}

// Origin (x0, y0) of the tile of work item b (after the XCD remap); thread
// (lx, ly) takes the nodes (x0 + lx, y0 + ly + j ty), j < rows.
__host__ __device__ inline void mc_tile_origin(int b, int nx, int tx, int ty, int rows, int &x0, int &y0)
{
    const int ntx = (nx + tx - 1) / tx;
    x0 = (b % ntx) * tx;
    y0 = (b / ntx) * ty * rows;
}

// LDS cell (lx, ly) of ring entry k of a tile's (LX x LY)-cell density plane:
// row 0, row LY - 1, then columns 0 and LX - 1 of the rows between
// (2 LX + 2 (LY - 2) entries in all).
__host__ __device__ inline void mc_ring_cell(int k, int LX, int LY, int &lx, int &ly)
{
    const int TYR = LY - 2;
    lx = k < 2 * LX ? k % LX : (k < 2 * LX + TYR ? 0 : LX - 1);
    ly = k < LX ? 0 : (k < 2 * LX ? LY - 1 : (k < 2 * LX + TYR ? k - 2 * LX + 1 : k - 2 * LX - TYR + 1));
}

hipError_t launch_step_mc(int precision, const StepMCArgs &a);

// Utility launches over the nodes of the run: op 0 = populations [2][9][N]
// into buf (FP64, host order), op 1 = populations from buf into fout, op 2 =
// equilibrium from buf = (rhoA, rhoB, ux, uy) [4][N] into fout, op 3 =
// densities [2][N] into buf, op 4 = Eq. (6) mixture velocity from the
// densities in buf[0..2N) into buf[2N..4N) (reads fin for the momenta).
hipError_t launch_util_mc(int precision, int op, const RunMC *run, const void *fin, void *fout, double *buf,
                          int64_t nodes, hipStream_t stream);
// Per-block FP64 partial sums of the drop diagnostics from buf = (rhoA, rhoB,
// ux, uy) [4][N]: 11 values per block (mass A, mass B, sum rhoA_in, sum
// rhoB_in, n_in, sum rhoA_out, sum rhoB_out, n_out, sum p_in, sum p_out, max |u|).
hipError_t launch_diag_mc(const RunMC *run, const double *buf, double cx, double cy, double r_in, double r_out,
                          double *partial, int64_t nodes, hipStream_t stream);
constexpr int kThreadsMC = 256;
constexpr int kDiagMC = 11;

} // namespace lbmmc
