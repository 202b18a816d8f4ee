// Launch interface of the D3Q19 kernels (lbm3d_kernels.hip), internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace lbm3 {

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
    hipStream_t stream;
    hipEvent_t ev_psi0 = nullptr, ev_psi1 = nullptr, ev_col0 = nullptr, ev_col1 = nullptr;
};

// psi pass then collide-and-push into fout (one time step).
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

} // namespace lbm3
