// vlb_aux.hip -- gfx950 kernels around the coupled step: equilibrium initial state,
// readout of rho, u and A, the monitors (deterministic two-pass reductions), and the
// small fill/header kernels the host uses instead of memset (safe under graph capture).
// The step kernels themselves live in vlb_kernels.hip.
#include "vlb_device.h"

namespace vlb {
namespace {

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
    T phi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) phi[k] = a[k] ? (T)a[k][q] : phi0(k);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (solid) {
            st4<false>(dst, plane, i, (unsigned)p, make4<S>(0.0, 0.0, 0.0, 0.0));
        } else {
            st4<false>(dst, plane, i, (unsigned)p,
                       make4<S>(dfeq(i, r - 1.0, r, vx, vy), dgeq(i, phi[0] - phi0(0), phi[0], vx, vy),
                                dgeq(i, phi[1] - phi0(1), phi[1], vx, vy),
                                dgeq(i, phi[2] - phi0(2), phi[2], vx, vy)));
        }
    }
    const T zero[3] = {0.0, 0.0, 0.0};
    hist_st<false>(R.hist, plane, (unsigned)p, zero, 0.0, 0.0);
}

// Macroscopic fields of node (x, y) at the current time; false for solid nodes.  At a
// wall-adjacent node phi is phi_b, which CNEBB keeps.
template <class S>
__device__ __forceinline__ bool node_fields(const RunDev<S>& R, const S* src, int x, int y,
                                            bool pull, T& rho, T& ux, T& uy, T a[3]) {
    const int p = node_index(R, x, y);
    const unsigned b = node_bits(R, p);
    if (b & BIT_SELF_SOLID) return false;
    S f[9], g[3][9];
    pull36(R, src, p, pull, f, g);
    if (pull && R.ylw && (b & 0x1FEu)) ylw_restore(R, src, p, b, f);
    T Fx, Fy, drho;
    node_force(R, p, Fx, Fy);
    const bool wet = wet_row(R, y);
    if (pull && nebb_end(R, x)) zou_he_x(f, x == 0, T(R.inlet[y]), Fx, Fy);
    if (wet && pull) zou_he(f, y == 0, Fx, Fy);
    hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
    if (wet) ux = uy = 0.0;  // wall node: the wall velocity
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T acc = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) acc += T(g[k][i]);
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

// History the next step uses (S(t-1) and u(t-1)), unpadded [ny][nx] arrays.
template <class S>
__global__ void k_read_history(const RunDev<S>* __restrict__ run, S* sxx, S* sxy, S* syy, S* uxp,
                               S* uyp) {
    const RunDev<S>& R = *run;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= R.nx || y >= R.ny) return;
    const int q = y * R.nx + x;
    T hS[3], hux, huy;
    hist_ld(R.hist, R.plane, (unsigned)node_index(R, x, y), hS, hux, huy);
    if (sxx) sxx[q] = (S)hS[0];
    if (sxy) sxy[q] = (S)hS[1];
    if (syy) syy[q] = (S)hS[2];
    if (uxp) uxp[q] = (S)hux;
    if (uyp) uyp[q] = (S)huy;
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

// Monitors: mass of each lattice (FP64), residual since the last snapshot, max |u|,
// non-finite and non-SPD counts.  Two deterministic passes: each block reduces its
// 4 x 64 nodes (wavefront shuffles, then the four waves in order) into 8 partials;
// one block then reduces the partials in a fixed order.
enum { MON_NPART = 8 };  // mass x 4, residual, umax, non-finite, non-SPD

template <class S>
__global__ __launch_bounds__(256) void k_monitor(const RunDev<S>* __restrict__ run, int parity,
                                                 int first, S* usnap, double* part) {
    __shared__ double s_p[4][MON_NPART];
    const RunDev<S>& R = *run;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    double v[MON_NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (x < R.nx && y < R.ny) {
        T r, vx, vy, a[3];
        if (node_fields(R, R.pop[parity], x, y, first == 0, r, vx, vy, a)) {
            const int q = y * R.nx + x;
            const bool ok = isfinite(r) && isfinite(vx) && isfinite(vy) && isfinite(a[0]) &&
                            isfinite(a[1]) && isfinite(a[2]);
            if (ok) {
                v[0] = r; v[1] = a[0]; v[2] = a[1]; v[3] = a[2];
                const double dx = vx - (double)usnap[q], dy = vy - (double)usnap[R.nx * R.ny + q];
                v[4] = sqrt(dx * dx + dy * dy);
                v[5] = sqrt(vx * vx + vy * vy);
                const double det = a[0] * a[2] - a[1] * a[1];
                v[7] = (det <= 0.0 || a[0] + a[2] <= 0.0) ? 1.0 : 0.0;
            } else {
                v[6] = 1.0;
            }
            usnap[q] = (S)vx;
            usnap[R.nx * R.ny + q] = (S)vy;
        }
    }
    for (int c = 0; c < MON_NPART; ++c) v[c] = (c == 4 || c == 5) ? wave_max(v[c]) : wave_sum(v[c]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < MON_NPART; ++c) s_p[w][c] = v[c];
    __syncthreads();
    if (threadIdx.x < MON_NPART) {
        const int c = threadIdx.x;
        double t = s_p[0][c];
        for (int k = 1; k < 4; ++k) t = (c == 4 || c == 5) ? fmax(t, s_p[k][c]) : t + s_p[k][c];
        part[(size_t)(blockIdx.y * gridDim.x + blockIdx.x) * MON_NPART + c] = t;
    }
}

__global__ __launch_bounds__(256) void k_monitor_final(const double* __restrict__ part, int nblocks,
                                                       MonitorAcc* acc) {
    __shared__ double s_p[4][MON_NPART];
    double v[MON_NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
        for (int c = 0; c < MON_NPART; ++c) {
            const double t = part[(size_t)b * MON_NPART + c];
            v[c] = (c == 4 || c == 5) ? fmax(v[c], t) : v[c] + t;
        }
    for (int c = 0; c < MON_NPART; ++c) v[c] = (c == 4 || c == 5) ? wave_max(v[c]) : wave_sum(v[c]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < MON_NPART; ++c) s_p[w][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[MON_NPART];
        for (int c = 0; c < MON_NPART; ++c) {
            t[c] = s_p[0][c];
            for (int k = 1; k < 4; ++k) t[c] = (c == 4 || c == 5) ? fmax(t[c], s_p[k][c]) : t[c] + s_p[k][c];
        }
        for (int c = 0; c < 4; ++c) acc->mass[c] = t[c];
        acc->residual = t[4];
        acc->umax = t[5];
        acc->nonfinite = (unsigned long long)t[6];
        acc->spd = (unsigned long long)t[7];
    }
}

// Momentum-exchange force on the solid (Sec. 4.3): per boundary link (fluid node x_f,
// direction d with x_f + e_d solid) e_d (f_d^post(x_f) + f_opp(d)(x_f, t + 1)); the buffer
// just written holds the post-collision values at the nodes and, in the slot x_f + e_d,
// the population the boundary rule returns.  Links of other circles contribute zero.
template <class S>
__global__ __launch_bounds__(256) void k_drag(const RunDev<S>* __restrict__ run,
                                              const int* __restrict__ links, int nlinks,
                                              int circle, int parity, double* part) {
    __shared__ double s_p[4][2];
    const RunDev<S>& R = *run;
    const int t = blockIdx.x * 256 + threadIdx.x;
    double fx = 0.0, fy = 0.0;
    if (t < nlinks) {
        const int p = links[3 * t], d = links[3 * t + 1], cid = links[3 * t + 2];
        if (circle < 0 || cid == circle) {
            const S* buf = R.pop[parity];
            const long long plane = R.plane;
            const int o = opp(d);
            const T v = ld1(buf, plane, 0, d, (unsigned)p) +
                        ld1(buf, plane, 0, o, (unsigned)(p + ex(d) + ey(d) * R.pitch)) + 2.0 * wgt(d);
            fx = T(ex(d)) * v;
            fy = T(ey(d)) * v;
        }
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_p[w][0] = fx;
        s_p[w][1] = fy;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int c = threadIdx.x;
        part[2 * blockIdx.x + c] = ((s_p[0][c] + s_p[1][c]) + s_p[2][c]) + s_p[3][c];
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
hipError_t launch_read_history(const RunDev<S>& h, const RunDev<S>* d, S* sxx, S* sxy, S* syy,
                               S* uxp, S* uyp, hipStream_t s) {
    dim3 blk(64, 4), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_read_history<S>), grd, blk, 0, s, d, sxx, sxy, syy, uxp, uyp);
    return hipGetLastError();
}

template <class S>
hipError_t launch_monitor(const RunDev<S>& h, const RunDev<S>* d, int parity, int first,
                          S* usnap, double* part, MonitorAcc* acc, hipStream_t s) {
    dim3 blk(256), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_monitor<S>), grd, blk, 0, s, d, parity, first, usnap, part);
    hipLaunchKernelGGL(k_monitor_final, dim3(1), blk, 0, s, (const double*)part,
                       (int)(grd.x * grd.y), acc);
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


template <class S>
hipError_t launch_drag(const RunDev<S>* run_dev, const int* links, int nlinks, int circle,
                       int parity, double* part, hipStream_t s) {
    if (nlinks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_drag<S>), dim3((nlinks + 255) / 256), dim3(256), 0, s, run_dev, links,
                       nlinks, circle, parity, part);
    return hipGetLastError();
}

#define VLB_INSTANTIATE_AUX(S)                                                               \
    template hipError_t launch_init<S>(const RunDev<S>&, const RunDev<S>*, const S*,       \
                                       const S*, const S*, const S*, const S*, const S*,  \
                                       hipStream_t);                                       \
    template hipError_t launch_read<S>(const RunDev<S>&, const RunDev<S>*, int, int, S*,   \
                                       S*, S*, S*, S*, S*, hipStream_t);                   \
    template hipError_t launch_read_history<S>(const RunDev<S>&, const RunDev<S>*, S*, S*, \
                                               S*, S*, S*, hipStream_t);                   \
    template hipError_t launch_monitor<S>(const RunDev<S>&, const RunDev<S>*, int, int,    \
                                          S*, double*, MonitorAcc*, hipStream_t);          \
    template hipError_t launch_drag<S>(const RunDev<S>*, const int*, int, int, int, double*, \
                                       hipStream_t);
VLB_INSTANTIATE_AUX(float)
VLB_INSTANTIATE_AUX(double)

}  // namespace vlb
