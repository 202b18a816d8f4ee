// Launch interface between the host runtime (lbm_api.hip) and the kernels
// (lbm_kernels.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

struct RunDev;
struct Tile;

enum : int { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2 };

// threads per tile of the step kernels: 64 to kMaxTileThreads
constexpr int kMaxTileThreads = 512;

// Everything one step launch needs.
struct StepArgs {
    const RunDev *runs;
    const Tile *tiles;
    int ntiles;
    int tx, ty;
    void *f;
    void *psi;
    int32_t *status;
    hipStream_t stream;
    int xcd = 1;                    // XCD-aware work-list order
    int fused = 0;                  // nodes per thread of the fused kernel (1, 2, 4; one kernel per step,
                                    // f -> f_alt); 0: two kernels per step, in place on f
    void *f_alt = nullptr;          // second population buffer of the fused schedule (FP64 / FP32)
    const Tile *ftiles = nullptr;   // work list of the fused kernel: tiles of tx x (fused ty) nodes
    int nftiles = 0;
    float *r0 = nullptr;            // writer densities of bf16 storage: a step of parity p
    float *r1 = nullptr;            // reads R[p ^ 1] and writes R[p] (r0 = R[0], r1 = R[1])
    uint32_t *seed = nullptr;       // rounding-seed counter pair, slot p written by step p
    int halo = 1;                   // psi halo of the collide tile: 2 when a run uses Eq. (9)
    hipEvent_t ev_start = nullptr;  // optional events around a single launch
    hipEvent_t ev_stop = nullptr;
};

enum : int { UTIL_INIT = 0, UTIL_PUT = 1, UTIL_GET = 2, UTIL_MOMENTS = 3, UTIL_COLUMN = 4, UTIL_PRESSURE = 5,
             UTIL_WINDOW = 6 };

// One utility launch over the nodes of a single run.
struct UtilArgs {
    int op;
    const RunDev *runs;
    int run;
    int64_t nodes;
    void *f;
    const void *psi;
    double *buf;      // INIT: rho; PUT: source f; GET: destination f; MOMENTS: rho, ux, uy; PRESSURE: p
    const double *ux; // INIT only (may be null)
    const double *uy; // INIT only (may be null)
    int parity;
    int index = 0;    // COLUMN: the column x
    int wx0 = 0, wy0 = 0, ww = 0, wh = 0; // WINDOW: origin (wrapped on periodic axes) and size
    float *r0 = nullptr, *r1 = nullptr; // bf16 writer densities (the current state uses R[parity ^ 1])
    hipStream_t stream;
};

hipError_t launch_step(int precision, const StepArgs &a, int parity);
hipError_t launch_collide(int precision, const StepArgs &a, int parity);
hipError_t launch_fused(int precision, const StepArgs &a, int parity);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t stream);
hipError_t launch_psi(int precision, const StepArgs &a, int parity);
hipError_t launch_util(int precision, const UtilArgs &u);
hipError_t launch_diag(int precision, const StepArgs &a, const double *regions, double *partial, double *out,
                       int nruns, int parity);
hipError_t launch_table_setup(const RunDev &r, RunDev *runs, Tile *tiles, int ntx, int ntiles, int tx, int ty,
                              int32_t *status, hipStream_t stream);

} // namespace lbm
