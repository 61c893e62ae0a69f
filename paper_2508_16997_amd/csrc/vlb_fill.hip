// Boundary fill: the second launch of every time step (after k_step).
//
// k_fill walks the run's list of boundary links -- one op per fluid node and direction
// whose pull source is neither a fluid node nor a periodic image -- and writes into
// that ghost or solid slot of the buffer just written the value the boundary rule
// gives: half-way bounce-back (walls, staircase solids) or linear interpolated
// bounce-back (curved links) for f, the wall-bound population for the conformation
// lattices (the input of CNEBB in the next step), and non-equilibrium extrapolation
// at the open ends (Sec. 4.3).  Every (slot, direction) pair belongs to one fluid
// node, so the ops never conflict; the host groups them by kind so that a wavefront
// runs one rule.
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
        // Open ends: non-equilibrium extrapolation from the node x0 next to the ghost
        // (first or last column, same row): its post-collision populations minus their
        // own equilibrium, plus the equilibrium of the boundary state -- inlet: rho(x0)
        // and the inlet profile (u_in, A_in); outlet: rho = 1 and u(x0) for the
        // hydrodynamic lattice, a plain copy of x0 for the conformation lattices.
        const bool in = kind == FILL_INLET;
        const int x0 = in ? R.off0 + op.far * R.pitch : op.src;
        const T uin = in ? T(R.inlet[op.far]) : 0.0;
        if (node_bits(R, x0) & BIT_SELF_SOLID) {
            stu(buf + dir * plane, (unsigned)op.dst, in ? dfeq(dir, 0.0, 1.0, uin, 0.0) : 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T a = in ? T(R.inlet[(1 + k) * R.ny + op.far]) : phi0(k);
                stu(buf + (9 + 9 * k + dir) * plane, (unsigned)op.dst,
                    in ? dgeq(dir, a - phi0(k), a, uin, 0.0) : 0.0);
            }
            return;
        }
        T d[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) d[j] = ldu(buf + j * plane, (unsigned)x0);
        T drho, rho, vx, vy;
        hydro_macros(d, 0.0, 0.0, drho, rho, vx, vy);
        const T fneq = d[dir] - dfeq(dir, drho, rho, vx, vy);
        stu(buf + dir * plane, (unsigned)op.dst,
            (in ? dfeq(dir, drho, rho, uin, 0.0) : dfeq(dir, 0.0, 1.0, vx, vy)) + fneq);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const S* pl = buf + (9 + 9 * k) * plane;
            if (!in) {
                stu(buf + (9 + 9 * k + dir) * plane, (unsigned)op.dst, ldu(pl + dir * plane, (unsigned)x0));
                continue;
            }
            T dphi = 0.0;
#pragma unroll
            for (int j = 0; j < 9; ++j) dphi += ldu(pl + j * plane, (unsigned)x0);
            const T a = R.inlet[(1 + k) * R.ny + op.far];
            stu(buf + (9 + 9 * k + dir) * plane, (unsigned)op.dst,
                dgeq(dir, a - phi0(k), a, uin, 0.0) + ldu(pl + dir * plane, (unsigned)x0) -
                    dgeq(dir, dphi, phi0(k) + dphi, vx, vy));
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
