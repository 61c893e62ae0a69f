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
    S* buf = R.pop[parity];
    const long long plane = R.plane;
    const int dir = op.dir_kind & 0xff, kind = op.dir_kind >> 8;
    const int o = opp(dir);
    if (kind == FILL_OUTLET || kind == FILL_INLET) {
        // Open-end ghosts whose extrapolation node x0 (first or last column, row `far`)
        // is solid: the equilibrium of the boundary state (inlet profile, or rest at the
        // outlet), constant in time.  Ghosts of fluid x0 are written by the step kernel
        // itself.
        const bool in = kind == FILL_INLET;
        const T uin = in ? T(R.inlet[op.far]) : 0.0;
        stu(buf + dir * plane, (unsigned)op.dst, in ? dfeq(dir, 0.0, 1.0, uin, 0.0) : 0.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T a = in ? T(R.inlet[(1 + k) * R.ny + op.far]) : phi0(k);
            stu(buf + (9 + 9 * k + dir) * plane, (unsigned)op.dst,
                in ? dgeq(dir, a - phi0(k), a, uin, 0.0) : 0.0);
        }
    } else {
        // conformation lattices: the population that left toward the wall (CNEBB input)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            stu(buf + (9 + 9 * k + dir) * plane, (unsigned)op.dst,
                ldu(buf + (9 + 9 * k + o) * plane, (unsigned)op.src));
        // hydrodynamic lattice: half-way or linear interpolated bounce-back
        const T fo = ldu(buf + o * plane, (unsigned)op.src);
        T v = fo;
        if (kind == FILL_CURVED) {
            const T q = op.q;
            if (q < 0.5) {
                if (op.far >= 0) v = 2.0 * q * fo + (1.0 - 2.0 * q) * ldu(buf + o * plane, (unsigned)op.far);
            } else {
                v = fo / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * ldu(buf + dir * plane, (unsigned)op.src);
            }
        }
        stu(buf + dir * plane, (unsigned)op.dst, v);
    }
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
