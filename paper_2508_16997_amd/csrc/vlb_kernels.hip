// vlb_kernels.hip -- gfx950 kernels of the coupled viscoelastic lattice Boltzmann step.
//
// Per time step two launches (pull scheme, two population buffers):
//   k_step  every lane pulls its node's 36 post-collision populations from the
//           neighbours' slots with one branch-free global load each (structure-of-
//           arrays planes, x fastest, 64 lanes read contiguous rows).  Slots that do
//           not hold a fluid node -- ghost rows/columns around the domain and solid
//           nodes -- were written by k_fill with exactly the value the boundary rule
//           gives for that link.  rho and u of the 64 x TY tile and of a one-node ring
//           around it go to LDS; then the velocity gradient and d(rho u^3) by finite
//           differences, CNEBB at wall-adjacent nodes, the constitutive source, the
//           hydrodynamic and three convection-diffusion collisions in moment form,
//           and 36 + 5 coalesced stores.
//   k_fill  walks the run's list of boundary links (one op per fluid node and
//           direction whose source is not a fluid node) and writes the periodic image,
//           the bounced or interpolated population, or the inlet equilibrium into the
//           slot that the next k_step pulls.  Every (slot, direction) pair belongs to
//           one fluid node, so the ops never conflict.
// Storage is float or double (template S); populations are kept as deviations from
// the rest state (f_i - w_i, g_i - w_i phi0 with phi0 = 1, 0, 1).  All arithmetic is
// double precision: on CDNA the vector FP64 rate equals the unpacked FP32 rate, and
// single-precision arithmetic lets rounding drift accumulate over many steps.
// The collision is the paper's regularized TRT operator rewritten in Hermite-moment
// space (algebraically identical to the per-direction form).
#include "vlb_device.h"

// Register budget of the step kernel: single-precision storage fits four waves per
// SIMD (a few spilled registers cost less than the lost latency hiding); double
// precision keeps its natural allocation.
template <class S, int TY>
struct StepBounds {
    static constexpr int threads = 64 * TY;
    static constexpr int min_waves_per_eu = sizeof(S) == 4 ? 4 : 1;
};

namespace vlb {
namespace {

template <class S, int TY, bool NT>
__global__ __launch_bounds__((StepBounds<S, TY>::threads), (StepBounds<S, TY>::min_waves_per_eu)) void k_step(
    const RunDev<S>* __restrict__ runs, const Item* __restrict__ items, int parity, int first) {
    __shared__ T s_rho[TY + 2][66];
    __shared__ T s_ux[TY + 2][66];
    __shared__ T s_uy[TY + 2][66];
    const Item it = items[blockIdx.x];
    const RunDev<S>& R = runs[it.run];
    const S* src = R.pop[parity];
    S* dst = R.pop[parity ^ 1];
    const long long plane = R.plane;
    const bool pull = first == 0;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * 64 + lx;
    const int x0 = it.tx * 64, y0 = it.ty * TY;
    const int x = x0 + lx, y = y0 + ly;

    // ---- phase 1: own node (36 pulls, history, force) ----
    const bool in_dom = x < R.nx && y < R.ny;
    const int p = node_index(R, x, y);
    unsigned b = 0u;
    if (in_dom) b = node_bits(R, p);
    const bool active = in_dom && !(b & BIT_SELF_SOLID);
    S f[9], g[3][9];
    T Fx = 0.0, Fy = 0.0, hS[3] = {0.0, 0.0, 0.0}, hux = 0.0, huy = 0.0;
    if (active) {
        pull9(R, src, 0, p, pull, f);
#pragma unroll
        for (int k = 0; k < 3; ++k) pull9(R, src, 1 + k, p, pull, g[k]);
        node_force(R, p, Fx, Fy);
        if (pull) {
#pragma unroll
            for (int k = 0; k < 3; ++k) hS[k] = ldu(R.hist + k * plane, (unsigned)p);
            hux = ldu(R.hist + 3 * plane, (unsigned)p);
            huy = ldu(R.hist + 4 * plane, (unsigned)p);
        }
    }
    // ring cells: rows above/below the tile, columns left/right of it
    for (int r = tid; r < 128 + 2 * TY; r += 64 * TY) {
        int cx, cy, lcx, lcy;
        if (r < 64) { cx = x0 + r; cy = y0 - 1; lcx = r + 1; lcy = 0; }
        else if (r < 128) { cx = x0 + r - 64; cy = y0 + TY; lcx = r - 63; lcy = TY + 1; }
        else if (r < 128 + TY) { cx = x0 - 1; cy = y0 + r - 128; lcx = 0; lcy = r - 127; }
        else { cx = x0 + 64; cy = y0 + r - 128 - TY; lcx = 65; lcy = r - 127 - TY; }
        T rr, vx, vy;
        if (cell_macros(R, src, cx, cy, pull, rr, vx, vy)) {
            s_rho[lcy][lcx] = rr;
            s_ux[lcy][lcx] = vx;
            s_uy[lcy][lcx] = vy;
        }
    }
    T drho = 0.0, rho = 1.0, ux = 0.0, uy = 0.0;
    if (active) {
        hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
        s_rho[ly + 1][lx + 1] = rho;
        s_ux[ly + 1][lx + 1] = ux;
        s_uy[ly + 1][lx + 1] = uy;
    } else if (!in_dom) {
        // out-of-domain tile cell: periodic image for the neighbours' differences
        T rr, vx, vy;
        if (cell_macros(R, src, x, y, pull, rr, vx, vy)) {
            s_rho[ly + 1][lx + 1] = rr;
            s_ux[ly + 1][lx + 1] = vx;
            s_uy[ly + 1][lx + 1] = vy;
        }
    }
    __syncthreads();
    if (!active) return;

    // ---- phase 2 ----
    // neighbour values for the differences: LDS for fluid neighbours, the wall formula
    // at walls, inlet/outlet ghost values at open ends.
    const bool wxl = (b >> 1) & 1u, wxh = (b >> 3) & 1u, wyl = (b >> 2) & 1u, wyh = (b >> 4) & 1u;
    T qxl = 0.5, qxh = 0.5, qyl = 0.5, qyh = 0.5;
    if (R.has_curved && (b & 0x1Eu)) {
        const int bi = R.bidx[p];
        qxl = link_q(R, bi, 1); qxh = link_q(R, bi, 3);
        qyl = link_q(R, bi, 2); qyh = link_q(R, bi, 4);
    }
    const bool open_l = R.xmode == XM_OPEN && x == 0;
    const bool open_h = R.xmode == XM_OPEN && x == R.nx - 1;
    T rl = 0.0, uxl = 0.0, uyl = 0.0, rh = 0.0, uxh = 0.0, uyh = 0.0;
    if (open_l) { rl = 1.0; uxl = R.inlet[y]; }
    else if (!wxl) { rl = s_rho[ly + 1][lx]; uxl = s_ux[ly + 1][lx]; uyl = s_uy[ly + 1][lx]; }
    if (open_h) { rh = rho; uxh = ux; uyh = uy; }
    else if (!wxh) { rh = s_rho[ly + 1][lx + 2]; uxh = s_ux[ly + 1][lx + 2]; uyh = s_uy[ly + 1][lx + 2]; }
    T rd = 0.0, uxd = 0.0, uyd = 0.0, ru = 0.0, uxu = 0.0, uyu = 0.0;
    if (!wyl) { rd = s_rho[ly][lx + 1]; uxd = s_ux[ly][lx + 1]; uyd = s_uy[ly][lx + 1]; }
    if (!wyh) { ru = s_rho[ly + 2][lx + 1]; uxu = s_ux[ly + 2][lx + 1]; uyu = s_uy[ly + 2][lx + 1]; }
    const T Lxx = dgrad(wxl, qxl, uxl, ux, wxh, qxh, uxh);
    const T Lxy = dgrad(wxl, qxl, uyl, uy, wxh, qxh, uyh);
    const T Lyx = dgrad(wyl, qyl, uxd, ux, wyh, qyh, uxu);
    const T Lyy = dgrad(wyl, qyl, uyd, uy, wyh, qyh, uyu);
    const T Dx = dgrad(wxl, qxl, rl * uxl * uxl * uxl, rho * ux * ux * ux, wxh, qxh,
                       rh * uxh * uxh * uxh);
    const T Dy = dgrad(wyl, qyl, rd * uyd * uyd * uyd, rho * uy * uy * uy, wyh, qyh,
                       ru * uyu * uyu * uyu);

    // conformation: CNEBB at wall-adjacent nodes, then the moments of each lattice
    const unsigned solid = pull ? (b & 0x1FEu) : 0u;
    Mom gm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (solid) {
            T gg[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) gg[i] = T(g[k][i]);
            cnebb(solid, k, ux, uy, gg);
            gm[k] = moments(gg);
        } else {
            gm[k] = moments(g[k]);
        }
    }
    const T d0 = gm[0].m0, d1 = gm[1].m0, d2 = gm[2].m0;
    const T axx = 1.0 + d0, axy = d1, ayy = 1.0 + d2;
    const T txx = R.eta_over_lam * d0, txy = R.eta_over_lam * d1, tyy = R.eta_over_lam * d2;
    T Sc[3];
    if (R.no_source) {
        Sc[0] = Sc[1] = Sc[2] = 0.0;
    } else {
        const T d = Lxx + Lyy;
        Sc[0] = -R.inv_lam * d0 + 2.0 * (axx * Lxx + axy * Lyx) + axx * d;
        Sc[1] = -R.inv_lam * d1 + axx * Lxy + axy * Lyy + axy * Lxx + ayy * Lyx + axy * d;
        Sc[2] = -R.inv_lam * d2 + 2.0 * (axy * Lxy + ayy * Lyy) + ayy * d;
    }
    if (!pull) {  // first step: F~(t - 1) := F~(t)
        hS[0] = Sc[0]; hS[1] = Sc[1]; hS[2] = Sc[2];
        hux = ux; huy = uy;
    }

    // Periodic images: an edge node also writes the populations that leave the domain
    // into the ghost slots its periodic neighbours pull from (no fill op needed).
    const bool px_per = R.xmode == XM_PERIODIC, py_per = R.ymode == XM_PERIODIC;
    const int gxo = (px_per && x == R.nx - 1) ? -R.nx : ((px_per && x == 0) ? R.nx : 0);
    const int gyo = (py_per && y == R.ny - 1) ? -R.ny : ((py_per && y == 0) ? R.ny : 0);
    const bool edge = (gxo | gyo) != 0;
    // ghost slot of direction i for this node, or -1: a population moving in direction
    // i leaves through the edge it points at
    auto ghost = [&](int i) -> int {
        const int sx = (gxo != 0 && ex(i) == (gxo < 0 ? 1 : -1)) ? gxo : 0;
        const int sy = (gyo != 0 && ey(i) == (gyo < 0 ? 1 : -1)) ? gyo : 0;
        if (sx == 0 && sy == 0) return -1;
        return p + sx + sy * R.pitch;
    };

    T out[9];
    collide_hydro(R, moments(f), rho, ux, uy, Fx, Fy, txx, txy, tyy, Dx, Dy, out);
#pragma unroll
    for (int i = 0; i < 9; ++i) st_stream<NT>(dst + i * plane, (unsigned)p, out[i]);
    if (edge) {
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int gs = ghost(i);
            if (gs >= 0) stu(dst + i * plane, (unsigned)gs, out[i]);
        }
    }
    const T inv_rho = 1.0 / rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T phi = phi0(k) + gm[k].m0;
        collide_cde(R, gm[k], phi, ux, uy, phi * inv_rho, Fx, Fy, Sc[k], hS[k], hux, huy, out);
#pragma unroll
        for (int i = 0; i < 9; ++i) st_stream<NT>(dst + (9 + 9 * k + i) * plane, (unsigned)p, out[i]);
        if (edge) {
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const int gs = ghost(i);
                if (gs >= 0) stu(dst + (9 + 9 * k + i) * plane, (unsigned)gs, out[i]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) st_stream<NT>(R.hist_out + k * plane, (unsigned)p, Sc[k]);
    st_stream<NT>(R.hist_out + 3 * plane, (unsigned)p, ux);
    st_stream<NT>(R.hist_out + 4 * plane, (unsigned)p, uy);
}

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
    if (kind == FILL_COPY) {
#pragma unroll
        for (int L = 0; L < 4; ++L) {
            S* pl = buf + (9 * L + dir) * plane;
            stu(pl, (unsigned)op.dst, ldu(pl, (unsigned)op.src));
        }
    } else if (kind == FILL_INLET) {
        const int row = op.far;
        const T uin = R.inlet[row];
        stu(buf + dir * plane, (unsigned)op.dst, dfeq(dir, 0.0, 1.0, uin, 0.0));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T a = R.inlet[(1 + k) * R.ny + row];
            stu(buf + (9 + 9 * k + dir) * plane, (unsigned)op.dst, dgeq(dir, a - phi0(k), a, uin, 0.0));
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

// Equilibrium initial state into buffer 0; history cleared.
template <class S>
__global__ void k_init(const RunDev<S>* __restrict__ run, const S* rho0, const S* ux0,
                       const S* uy0, const S* a0, const S* a1, const S* a2) {
    const RunDev<S>& R = *run;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= R.nx || y >= R.ny) return;
    const int p = node_index(R, x, y);
    const int q = y * R.nx + x;
    const long long plane = R.plane;
    S* dst = R.pop[0];
    const bool solid = node_bits(R, p) & BIT_SELF_SOLID;
    const T r = rho0 ? (T)rho0[q] : 1.0;
    const T vx = ux0 ? (T)ux0[q] : 0.0, vy = uy0 ? (T)uy0[q] : 0.0;
    const S* a[3] = {a0, a1, a2};
#pragma unroll
    for (int i = 0; i < 9; ++i) stu(dst + i * plane, (unsigned)p, solid ? 0.0 : dfeq(i, r - 1.0, r, vx, vy));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T phi = a[k] ? (T)a[k][q] : phi0(k);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            stu(dst + (9 + 9 * k + i) * plane, (unsigned)p,
                solid ? 0.0 : dgeq(i, phi - phi0(k), phi, vx, vy));
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) stu(R.hist + c * plane, (unsigned)p, 0.0);
}

// Macroscopic fields of node (x, y) at the current time; false for solid nodes.  At a
// wall-adjacent node phi is phi_b, which CNEBB keeps.
template <class S>
__device__ __forceinline__ bool node_fields(const RunDev<S>& R, const S* src, int x, int y,
                                            bool pull, T& rho, T& ux, T& uy, T a[3]) {
    const int p = node_index(R, x, y);
    if (node_bits(R, p) & BIT_SELF_SOLID) return false;
    S f[9];
    pull9(R, src, 0, p, pull, f);
    T Fx, Fy, drho;
    node_force(R, p, Fx, Fy);
    hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        S g[9];
        pull9(R, src, 1 + k, p, pull, g);
        T acc = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) acc += T(g[i]);
        a[k] = phi0(k) + acc;
    }
    return true;
}

template <class S>
__global__ void k_read(const RunDev<S>* __restrict__ run, int parity, int first, S* rho_o, S* ux_o,
                       S* uy_o, S* axx_o, S* axy_o, S* ayy_o) {
    const RunDev<S>& R = *run;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= R.nx || y >= R.ny) return;
    const int q = y * R.nx + x;
    T r = 0.0, vx = 0.0, vy = 0.0, a[3] = {0.0, 0.0, 0.0};
    if (!node_fields(R, R.pop[parity], x, y, first == 0, r, vx, vy, a)) r = 0.0;
    if (rho_o) rho_o[q] = (S)r;
    if (ux_o) ux_o[q] = (S)vx;
    if (uy_o) uy_o[q] = (S)vy;
    if (axx_o) axx_o[q] = (S)a[0];
    if (axy_o) axy_o[q] = (S)a[1];
    if (ayy_o) ayy_o[q] = (S)a[2];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
    // non-negative doubles order like their bit patterns as unsigned integers
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// Monitors: mass of each lattice (FP64), residual since the last snapshot, max |u|,
// non-finite and non-SPD counts; wavefront shuffles then one atomic per wavefront.
template <class S>
__global__ __launch_bounds__(256) void k_monitor(const RunDev<S>* __restrict__ run, int parity,
                                                 int first, S* usnap, MonitorAcc* acc) {
    const RunDev<S>& R = *run;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    double m[4] = {0, 0, 0, 0}, res = 0, umax = 0, nf = 0, spd = 0;
    if (x < R.nx && y < R.ny) {
        T r, vx, vy, a[3];
        if (node_fields(R, R.pop[parity], x, y, first == 0, r, vx, vy, a)) {
            const int q = y * R.nx + x;
            const bool ok = isfinite(r) && isfinite(vx) && isfinite(vy) && isfinite(a[0]) &&
                            isfinite(a[1]) && isfinite(a[2]);
            if (ok) {
                m[0] = r; m[1] = a[0]; m[2] = a[1]; m[3] = a[2];
                const double dx = vx - (double)usnap[q], dy = vy - (double)usnap[R.nx * R.ny + q];
                res = sqrt(dx * dx + dy * dy);
                umax = sqrt(vx * vx + vy * vy);
                const double det = a[0] * a[2] - a[1] * a[1];
                spd = (det <= 0.0 || a[0] + a[2] <= 0.0) ? 1.0 : 0.0;
            } else {
                nf = 1.0;
            }
            usnap[q] = (S)vx;
            usnap[R.nx * R.ny + q] = (S)vy;
        }
    }
    for (int c = 0; c < 4; ++c) m[c] = wave_sum(m[c]);
    nf = wave_sum(nf);
    spd = wave_sum(spd);
    res = wave_max(res);
    umax = wave_max(umax);
    if ((threadIdx.x & 63) == 0) {
        for (int c = 0; c < 4; ++c) atomicAdd(&acc->mass[c], m[c]);
        atomic_max_nonneg(&acc->residual, res);
        atomic_max_nonneg(&acc->umax, umax);
        atomicAdd(&acc->nonfinite, (unsigned long long)nf);
        atomicAdd(&acc->spd, (unsigned long long)spd);
    }
}

__global__ void k_fill_bytes(unsigned char* dst, size_t n, unsigned char v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

__global__ void k_write_words(unsigned long long* dst, unsigned long long w0,
                              unsigned long long w1, unsigned long long w2,
                              unsigned long long w3) {
    if (threadIdx.x == 0) {
        dst[0] = w0;
        dst[1] = w1;
        dst[2] = w2;
        dst[3] = w3;
    }
}

}  // namespace

template <class S, bool NT>
hipError_t launch_step_nt(const RunDev<S>* runs_dev, const Item* items_dev, int nitems, int ty,
                          int parity, int first, hipStream_t s) {
    switch (ty) {
        case 1: hipLaunchKernelGGL((k_step<S, 1, NT>), dim3(nitems), dim3(64, 1), 0, s, runs_dev, items_dev, parity, first); break;
        case 2: hipLaunchKernelGGL((k_step<S, 2, NT>), dim3(nitems), dim3(64, 2), 0, s, runs_dev, items_dev, parity, first); break;
        case 4: hipLaunchKernelGGL((k_step<S, 4, NT>), dim3(nitems), dim3(64, 4), 0, s, runs_dev, items_dev, parity, first); break;
        case 8: hipLaunchKernelGGL((k_step<S, 8, NT>), dim3(nitems), dim3(64, 8), 0, s, runs_dev, items_dev, parity, first); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S>
hipError_t launch_step(const RunDev<S>* runs_dev, const Item* items_dev, int nitems, int ty,
                       int parity, int first, int streaming, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    return streaming ? launch_step_nt<S, true>(runs_dev, items_dev, nitems, ty, parity, first, s)
                     : launch_step_nt<S, false>(runs_dev, items_dev, nitems, ty, parity, first, s);
}

template <class S>
hipError_t launch_fill(const RunDev<S>* runs_dev, const FillItem* items_dev, int nitems, int parity,
                       hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill<S>), dim3(nitems), dim3(256), 0, s, runs_dev, items_dev, parity);
    return hipGetLastError();
}

template <class S>
hipError_t launch_init(const RunDev<S>& h, const RunDev<S>* d, const S* rho, const S* ux,
                       const S* uy, const S* axx, const S* axy, const S* ayy, hipStream_t s) {
    dim3 blk(64, 4), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_init<S>), grd, blk, 0, s, d, rho, ux, uy, axx, axy, ayy);
    return hipGetLastError();
}

template <class S>
hipError_t launch_read(const RunDev<S>& h, const RunDev<S>* d, int parity, int first, S* rho,
                       S* ux, S* uy, S* axx, S* axy, S* ayy, hipStream_t s) {
    dim3 blk(64, 4), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_read<S>), grd, blk, 0, s, d, parity, first, rho, ux, uy, axx, axy, ayy);
    return hipGetLastError();
}

template <class S>
hipError_t launch_monitor(const RunDev<S>& h, const RunDev<S>* d, int parity, int first,
                          S* usnap, MonitorAcc* acc, hipStream_t s) {
    dim3 blk(256), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_monitor<S>), grd, blk, 0, s, d, parity, first, usnap, acc);
    return hipGetLastError();
}

hipError_t launch_fill_bytes(void* dst, size_t bytes, unsigned char v, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((bytes + 255) / 256);
    hipLaunchKernelGGL(k_fill_bytes, dim3(blocks), dim3(256), 0, s, (unsigned char*)dst, bytes, v);
    return hipGetLastError();
}

hipError_t launch_write_words(unsigned long long* dst, unsigned long long w0,
                              unsigned long long w1, unsigned long long w2,
                              unsigned long long w3, hipStream_t s) {
    hipLaunchKernelGGL(k_write_words, dim3(1), dim3(64), 0, s, dst, w0, w1, w2, w3);
    return hipGetLastError();
}

#define VLB_INSTANTIATE(S)                                                                   \
    template hipError_t launch_step<S>(const RunDev<S>*, const Item*, int, int, int, int,  \
                                       int, hipStream_t);                                  \
    template hipError_t launch_fill<S>(const RunDev<S>*, const FillItem*, int, int,        \
                                       hipStream_t);                                       \
    template hipError_t launch_init<S>(const RunDev<S>&, const RunDev<S>*, const S*,       \
                                       const S*, const S*, const S*, const S*, const S*,  \
                                       hipStream_t);                                       \
    template hipError_t launch_read<S>(const RunDev<S>&, const RunDev<S>*, int, int, S*,   \
                                       S*, S*, S*, S*, S*, hipStream_t);                   \
    template hipError_t launch_monitor<S>(const RunDev<S>&, const RunDev<S>*, int, int,    \
                                          S*, MonitorAcc*, hipStream_t);
VLB_INSTANTIATE(float)
VLB_INSTANTIATE(double)

}  // namespace vlb
