// Boundary fill: the second launch of every time step (after k_step).
//
// k_fill walks the run's list of boundary links -- one op per fluid node and direction
// whose pull source is a solid or a ghost not written by the step kernel -- and writes
// into that ghost or solid slot of the buffer just written the value the boundary rule
// gives: half-way bounce-back (walls, staircase solids) or linear interpolated
// bounce-back (curved links) for f, the wall-bound population for the conformation
// lattices (the input of CNEBB in the next step), and the constant equilibrium ghosts
// of open ends whose extrapolation node is solid.  (Periodic images and the open-end
// extrapolation from fluid nodes are stored by the step kernel.)  Every (slot,
// direction) pair belongs to one fluid node, so the ops never conflict; the host
// groups them by kind so that a wavefront runs one rule.
#include "vlb_device.h"

namespace vlb {
namespace {

// Boundary links of the buffer just written: write into each ghost or solid slot the
// value its fluid neighbour pulls in the next step.
template <class S>
__global__ __launch_bounds__(256) void k_fill(const RunDev<S>* __restrict__ runs,
                                              const FillItem* __restrict__ items, int parity) {
    const FillItem it = items[blockIdx.x];
    if ((int)threadIdx.x >= it.count) return;
    const RunDev<S>& R = runs[it.run];
    const FillOp op = R.fill[it.first + threadIdx.x];
    apply_fill_op(R, op, R.pop[parity]);
}

}  // namespace

template <class S>
hipError_t launch_fill(const RunDev<S>* runs_dev, const FillItem* items_dev, int nitems, int parity,
                       hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill<S>), dim3(nitems), dim3(256), 0, s, runs_dev, items_dev, parity);
    return hipGetLastError();
}

template hipError_t launch_fill<float>(const RunDev<float>*, const FillItem*, int, int, hipStream_t);
template hipError_t launch_fill<double>(const RunDev<double>*, const FillItem*, int, int, hipStream_t);

}  // namespace vlb
