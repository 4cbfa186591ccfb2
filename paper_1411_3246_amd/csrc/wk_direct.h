// Host-side interface of the Eq. (6)-direct response (wk_direct.hip).
#pragma once

#include "wk_internal.h"

namespace wk {

// Plasma response with B_theta from Eq. (6) as written (wk_direct.hip): FP64,
// one workgroup, Newton-GMRES per slice on the implicit d_xi E_z.
constexpr int kDirectKrylov = 40;   // Krylov vectors per Newton step
struct DirectDesc {
    MarchDesc march;        // FP64 plasma, group 1
    double* ys;             // [4][np] trial predicted state (x, y, px, py)
    double* yn;             // [4][np] trial corrected state
    double* f0;             // [4][np] stage-1 derivative of the trial
    double* V;              // [kDirectKrylov + 1][stride] Krylov basis
    int32_t iters;          // Newton steps at most per slice
    double tol;             // stop when max |Phi(B) - B| <= tol max |Phi(B)|
    int32_t* iterations;    // optional: [n_xi] Newton steps used
};
size_t direct_lds_bytes(int n_nodes);
size_t direct_ws_doubles(int64_t np, int n_nodes);
hipError_t launch_march_direct(const DirectDesc& dd, hipStream_t s);

}  // namespace wk
