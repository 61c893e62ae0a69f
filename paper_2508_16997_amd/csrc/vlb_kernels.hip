// vlb_kernels.hip -- the per-step launch of the coupled viscoelastic lattice Boltzmann
// step: one workgroup per 64 x TY tile of the XCD-ordered work list (the tile body is in
// vlb_step.h); the boundary fill list follows as its own launch (vlb_fill.hip).
#include "vlb_step.h"

namespace vlb {
namespace {

template <class S, int TY, bool NT, int W>
__global__ __launch_bounds__((StepBounds<S, TY, W>::threads), (StepBounds<S, TY, W>::min_waves_per_eu)) void k_step(
    const RunDev<S>* __restrict__ runs, const Item* __restrict__ items, int parity, int first) {
    step_tile<S, TY, NT>(runs, items[blockIdx.x], parity, first, 0);
}

}  // namespace

template <class S, bool NT, int W>
hipError_t launch_step_w(const RunDev<S>* runs_dev, const Item* items_dev, int nitems, int ty,
                         int parity, int first, hipStream_t s) {
    switch (ty) {
        case 1: hipLaunchKernelGGL((k_step<S, 1, NT, W>), dim3(nitems), dim3(64, 1), 0, s, runs_dev, items_dev, parity, first); break;
        case 2: hipLaunchKernelGGL((k_step<S, 2, NT, W>), dim3(nitems), dim3(64, 2), 0, s, runs_dev, items_dev, parity, first); break;
        case 4: hipLaunchKernelGGL((k_step<S, 4, NT, W>), dim3(nitems), dim3(64, 4), 0, s, runs_dev, items_dev, parity, first); break;
        case 8: hipLaunchKernelGGL((k_step<S, 8, NT, W>), dim3(nitems), dim3(64, 8), 0, s, runs_dev, items_dev, parity, first); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S, bool NT>
hipError_t launch_step_nt(const RunDev<S>* runs_dev, const Item* items_dev, int nitems, int ty,
                          int parity, int first, int waves, hipStream_t s) {
    // the register budget matters for single-precision storage only (double precision
    // runs at its natural allocation whatever W says)
    if (sizeof(S) == 4 && waves == 4)
        return launch_step_w<S, NT, 4>(runs_dev, items_dev, nitems, ty, parity, first, s);
    return launch_step_w<S, NT, 3>(runs_dev, items_dev, nitems, ty, parity, first, s);
}

template <class S>
hipError_t launch_step(const RunDev<S>* runs_dev, const Item* items_dev, int nitems, int ty,
                       int parity, int first, int streaming, int waves, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    return streaming ? launch_step_nt<S, true>(runs_dev, items_dev, nitems, ty, parity, first, waves, s)
                     : launch_step_nt<S, false>(runs_dev, items_dev, nitems, ty, parity, first, waves, s);
}

template hipError_t launch_step<float>(const RunDev<float>*, const Item*, int, int, int, int, int,
                                       int, hipStream_t);
template hipError_t launch_step<double>(const RunDev<double>*, const Item*, int, int, int, int,
                                        int, int, hipStream_t);

}  // namespace vlb
