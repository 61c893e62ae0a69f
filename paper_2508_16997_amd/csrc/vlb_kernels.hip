// vlb_kernels.hip -- gfx950 kernels of the coupled viscoelastic lattice Boltzmann step.
//
// One fused kernel per time step (pull scheme, two population buffers):
//   phase 1  every lane pulls its node's 36 post-collision populations from the
//            neighbours (one load each, structure-of-arrays planes, x fastest, so a
//            wavefront of 64 lanes reads contiguous rows), fills wall links
//            (half-way or linear interpolated bounce-back for f, the wall-bound
//            post-collision populations for g), and computes rho and u; a one-node
//            ring around the 64 x TY tile recomputes rho and u of its nodes from
//            their hydrodynamic populations only.  rho, u of tile and ring go to LDS.
//   phase 2  velocity gradient and d(rho u^3) by finite differences from LDS,
//            CNEBB at boundary nodes, constitutive source, the hydrodynamic and three
//            convection-diffusion collisions in moment form, and 36 + 5 coalesced
//            stores to the other buffer.
// Populations are stored as deviations from the rest state (f_i - w_i,
// g_i - w_i phi0 with phi0 = 1, 0, 1) so that single precision keeps the small
// velocity and stress signals; the collision is the paper's regularized TRT
// operator rewritten in Hermite-moment space (algebraically identical).
#include "vlb_internal.h"

namespace vlb {
namespace {

// D2Q9 velocities in the paper's order (Sec. 3.1), their opposites and weights.
__host__ __device__ constexpr int ex(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
template <class T>
__device__ __forceinline__ constexpr T wgt(int i) {
    return i == 0 ? T(4.0 / 9.0) : (i <= 4 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}
template <class T>
__device__ __forceinline__ constexpr T third() { return T(1.0 / 3.0); }

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp");

// Per-node pull sources: element index of x - e_i (or the node itself for wall links),
// the inlet row for inlet links.
struct Srcs {
    int idx[9];
    unsigned solid;  // bit i: wall link (source solid)
    unsigned inl;    // bit i: source is the inlet ghost column
};

template <class T>
__device__ __forceinline__ void node_srcs(const RunDev<T>& R, int px, int py, unsigned b,
                                          bool pull, Srcs& s) {
    const int p = py * R.pitch + px;
    s.solid = pull ? (b & 0x1FEu) : 0u;
    s.inl = 0u;
    s.idx[0] = p;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (!pull || ((s.solid >> i) & 1u)) {
            s.idx[i] = p;
            continue;
        }
        int xs = px - ex(i), ys = py - ey(i);
        // Domain walls are flagged in the geometry bits, so only periodic wraps remain.
        if (ys < 0) ys += R.ny;
        else if (ys >= R.ny) ys -= R.ny;
        if (xs < 0) {
            if (R.xmode == XM_OPEN) {
                s.inl |= 1u << i;
                s.idx[i] = ys;
                continue;
            }
            xs += R.nx;
        } else if (xs >= R.nx) {
            xs = (R.xmode == XM_OPEN) ? R.nx - 1 : xs - R.nx;  // outlet: zero gradient
        }
        s.idx[i] = ys * R.pitch + xs;
    }
}

// Deviation of the third-order Hermite hydrodynamic equilibrium (Sec. 3.1):
// f_i^eq - w_i = w_i [drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u + 13.5 h3_i(u))].
template <class T>
__device__ __forceinline__ T dfeq(int i, T drho, T rho, T ux, T uy) {
    const T eu = T(ex(i)) * ux + T(ey(i)) * uy;
    const T hxxy = (T(ex(i) * ex(i)) - third<T>()) * T(ey(i));
    const T hxyy = (T(ey(i) * ey(i)) - third<T>()) * T(ex(i));
    const T h3 = hxxy * ux * ux * uy + hxyy * ux * uy * uy;
    return wgt<T>(i) * (drho + rho * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * (ux * ux + uy * uy) +
                                      T(13.5) * h3));
}

// Deviation of the second-order convection-diffusion equilibrium (Sec. 3.2).
template <class T>
__device__ __forceinline__ T dgeq(int i, T dphi, T phi, T ux, T uy) {
    const T eu = T(ex(i)) * ux + T(ey(i)) * uy;
    return wgt<T>(i) * (dphi + phi * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * (ux * ux + uy * uy)));
}

template <class T>
__device__ __forceinline__ T phi0(int k) { return k == 1 ? T(0) : T(1); }

// Wall fill of the hydrodynamic population moving in direction i into node p whose
// source is solid: half-way bounce-back for q = 1/2, linear interpolated bounce-back
// otherwise (q is the wall fraction of the link from p toward the solid).
template <class T>
__device__ __noinline__ T wall_fill_curved(const RunDev<T>& R, const T* __restrict__ src, int px,
                                           int py, int p, int i, T q) {
    const long long plane = R.plane;
    const int o = opp(i);
    const T fo = src[o * plane + p];
    if (q < T(0.5)) {
        int xf = px + ex(i), yf = py + ey(i);
        bool ok = true;
        if (yf < 0 || yf >= R.ny) {
            if (R.ymode == XM_PERIODIC) yf = yf < 0 ? yf + R.ny : yf - R.ny;
            else ok = false;
        }
        if (xf < 0 || xf >= R.nx) {
            if (R.xmode == XM_PERIODIC) xf = xf < 0 ? xf + R.nx : xf - R.nx;
            else ok = false;
        }
        if (ok && R.has_bits) ok = (R.bits[yf * R.pitch + xf] & BIT_SELF_SOLID) == 0;
        if (!ok) return fo;
        return T(2) * q * fo + (T(1) - T(2) * q) * src[o * plane + yf * R.pitch + xf];
    }
    return fo / (T(2) * q) + (T(2) * q - T(1)) / (T(2) * q) * src[i * plane + p];
}

template <class T>
__device__ __forceinline__ T link_q(const RunDev<T>& R, int bi, int i) {
    return bi >= 0 ? R.bq[bi * 8 + (i - 1)] : T(0.5);
}

// Pulled (and wall-filled) hydrodynamic populations of node (px, py).
template <class T>
__device__ __forceinline__ void load_hydro(const RunDev<T>& R, const T* __restrict__ src, int px,
                                           int py, const Srcs& s, int bi, T f[9]) {
    const long long plane = R.plane;
    const int p = py * R.pitch + px;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if ((s.solid >> i) & 1u) {
            const T q = link_q(R, bi, i);
            if (q == T(0.5)) f[i] = src[opp(i) * plane + p];
            else f[i] = wall_fill_curved(R, src, px, py, p, i, q);
        } else if ((s.inl >> i) & 1u) {
            const T uin = R.inlet[s.idx[i]];
            f[i] = dfeq<T>(i, T(0), T(1), uin, T(0));
        } else {
            f[i] = src[i * plane + s.idx[i]];
        }
    }
}

// Pulled conformation populations of lattice k; wall links take the post-collision
// population that left toward the wall (input of the CNEBB phi_b).
template <class T>
__device__ __forceinline__ void load_cde(const RunDev<T>& R, const T* __restrict__ src, int k,
                                         int p, const Srcs& s, T g[9]) {
    const long long plane = R.plane;
    const T* __restrict__ base = src + (long long)(9 + 9 * k) * plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if ((s.solid >> i) & 1u) {
            g[i] = base[opp(i) * plane + p];
        } else if ((s.inl >> i) & 1u) {
            const int row = s.idx[i];
            const T uin = R.inlet[row];
            const T a = R.inlet[(1 + k) * R.ny + row];
            g[i] = dgeq<T>(i, a - phi0<T>(k), a, uin, T(0));
        } else {
            g[i] = base[i * plane + s.idx[i]];
        }
    }
}

template <class T>
__device__ __forceinline__ void node_force(const RunDev<T>& R, int p, T& Fx, T& Fy) {
    if (R.uniform_force) {
        Fx = R.Fx;
        Fy = R.Fy;
    } else {
        Fx = R.force[p];
        Fy = R.force[R.plane + p];
    }
}

// rho, u with the half-force shift (Sec. 3.1).
template <class T>
__device__ __forceinline__ void hydro_macros(const T f[9], T Fx, T Fy, T& drho, T& rho, T& ux,
                                             T& uy) {
    T s = T(0), jx = T(0), jy = T(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        s += f[i];
        if (ex(i) != 0) jx += T(ex(i)) * f[i];
        if (ey(i) != 0) jy += T(ey(i)) * f[i];
    }
    drho = s;
    rho = T(1) + s;
    ux = (jx + T(0.5) * Fx) / rho;
    uy = (jy + T(0.5) * Fy) / rho;
}

// Conservative non-equilibrium bounce-back for one lattice at a boundary node
// (Sec. 3.3).  On entry g holds the known post-streaming populations and, on wall
// links, the post-collision populations that moved toward the wall; phi_b is their
// sum.  Unknowns are rebuilt from the equilibrium at (phi_b, u_b) plus the
// non-equilibrium part of the known opposite population (the equilibrium alone when
// the opposite is unknown too); g_0 restores phi_b exactly.
template <class T>
__device__ __forceinline__ void cnebb(unsigned solid, int k, T ux, T uy, T g[9], T& dphi) {
    T sum = T(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) sum += g[i];
    dphi = sum;
    const T phi = phi0<T>(k) + sum;
    T known[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) known[i] = g[i];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (!((solid >> i) & 1u)) continue;
        const int o = opp(i);
        T v = dgeq<T>(i, sum, phi, ux, uy);
        if (!((solid >> o) & 1u)) v += known[o] - dgeq<T>(o, sum, phi, ux, uy);
        g[i] = v;
    }
    T rest = sum;
#pragma unroll
    for (int i = 1; i < 9; ++i) rest -= g[i];
    g[0] = rest;
}

// Finite-difference derivative along one axis: central difference, or the quadratic
// through the no-slip wall value 0 at fraction q when a neighbour is a wall.
template <class T>
__device__ __forceinline__ T dgrad(bool lo_wall, T qlo, T vlo, T v0, bool hi_wall, T qhi, T vhi) {
    if (!lo_wall && !hi_wall) return T(0.5) * (vhi - vlo);
    if (lo_wall && !hi_wall) return qlo / (T(1) + qlo) * vhi + (T(1) - qlo) / qlo * v0;
    if (!lo_wall) return -(qhi / (T(1) + qhi) * vlo + (T(1) - qhi) / qhi * v0);
    return v0 * (qhi - qlo) / (qlo * qhi);
}

// Hydrodynamic TRT regularized collision in Hermite-moment form (Sec. 3.1): the
// post-collision populations are w_i [drho + 3 e.M1 + 4.5 H2:M2 + 13.5 H3:M3] with
//   M1 = rho u + (1 - 1/tau_s1) a_1 + (1 - 1/(2 tau_s1)) F                      (F_i)
//   M2 = rho uu + (1 - 1/tau_s1) a_2 - (1 - 1/(2 tau_s1)) diag(Dx, Dy) - tau/tau_s1
//        (G_i and T_i)
//   M3 = rho uuu + (1 - 1/tau_s2) a_3   (xxy and xyy; H_xxx = H_yyy = 0 on D2Q9)
// where a_n are the off-equilibrium Hermite moments of f (a_0 = 0 identically).
template <class T>
__device__ __forceinline__ void collide_hydro(const RunDev<T>& R, const T f[9], T drho, T rho,
                                              T ux, T uy, T Fx, T Fy, T txx, T txy, T tyy,
                                              T Dx, T Dy, T out[9]) {
    T jx = T(0), jy = T(0), pxx = T(0), pyy = T(0), pxy = T(0), qxxy = T(0), qxyy = T(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int cx = ex(i), cy = ey(i);
        if (cx != 0) { jx += T(cx) * f[i]; pxx += f[i]; }
        if (cy != 0) { jy += T(cy) * f[i]; pyy += f[i]; }
        if (cx != 0 && cy != 0) {
            pxy += T(cx * cy) * f[i];
            qxxy += T(cy) * f[i];
            qxyy += T(cx) * f[i];
        }
    }
    const T r3 = third<T>();
    const T ruxx = rho * ux * ux, ruyy = rho * uy * uy, ruxy = rho * ux * uy;
    const T ax = jx - rho * ux, ay = jy - rho * uy;
    const T axx = pxx - r3 * drho - ruxx;
    const T ayy = pyy - r3 * drho - ruyy;
    const T axy = pxy - ruxy;
    const T axxy = qxxy - r3 * jy - ruxx * uy;
    const T axyy = qxyy - r3 * jx - ruyy * ux;
    const T m1x = rho * ux + R.c1 * ax + R.h1 * Fx;
    const T m1y = rho * uy + R.c1 * ay + R.h1 * Fy;
    const T m2xx = ruxx + R.c1 * axx - R.h1 * Dx - R.inv_ts1 * txx;
    const T m2yy = ruyy + R.c1 * ayy - R.h1 * Dy - R.inv_ts1 * tyy;
    const T m2xy = ruxy + R.c1 * axy - R.inv_ts1 * txy;
    const T m3xxy = ruxx * uy + R.c2 * axxy;
    const T m3xyy = ruyy * ux + R.c2 * axyy;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int cx = ex(i), cy = ey(i);
        const T hxx = T(cx * cx) - r3, hyy = T(cy * cy) - r3;
        T v = drho + T(3) * (T(cx) * m1x + T(cy) * m1y) +
              T(4.5) * (hxx * m2xx + hyy * m2yy + T(2 * cx * cy) * m2xy);
        if (cx != 0 || cy != 0) v += T(13.5) * (hxx * T(cy) * m3xxy + hyy * T(cx) * m3xyy);
        out[i] = wgt<T>(i) * v;
    }
}

// Convection-diffusion TRT regularized collision in moment form (Sec. 3.2):
// w_i [dphi + 1.5 S - 0.5 S_prev + 3 e.N1 + 4.5 H2:N2] with
//   N1 = phi u + (1 - 1/tau_p1) b_1 + (1 - 1/(2 tau_p1)) (F phi/rho + 1.5 S u - 0.5 S_prev u_prev)
//   N2 = phi uu + (1 - 1/tau_p2) b_2,
// i.e. the equilibrium, the regularized non-equilibrium part, G~_i, F~_i and half the
// backward time difference of F~_i.
template <class T>
__device__ __forceinline__ void collide_cde(const RunDev<T>& R, const T g[9], T dphi, T phi, T ux,
                                            T uy, T fr, T Fx, T Fy, T S, T Sp, T uxp, T uyp,
                                            T out[9]) {
    T mx = T(0), my = T(0), pxx = T(0), pyy = T(0), pxy = T(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int cx = ex(i), cy = ey(i);
        if (cx != 0) { mx += T(cx) * g[i]; pxx += g[i]; }
        if (cy != 0) { my += T(cy) * g[i]; pyy += g[i]; }
        if (cx != 0 && cy != 0) pxy += T(cx * cy) * g[i];
    }
    const T r3 = third<T>();
    const T bx = mx - phi * ux, by = my - phi * uy;
    const T bxx = pxx - r3 * dphi - phi * ux * ux;
    const T byy = pyy - r3 * dphi - phi * uy * uy;
    const T bxy = pxy - phi * ux * uy;
    const T s0 = dphi + T(1.5) * S - T(0.5) * Sp;
    const T n1x = phi * ux + R.p1 * bx + R.h2 * (Fx * fr + T(1.5) * S * ux - T(0.5) * Sp * uxp);
    const T n1y = phi * uy + R.p1 * by + R.h2 * (Fy * fr + T(1.5) * S * uy - T(0.5) * Sp * uyp);
    const T n2xx = phi * ux * ux + R.p2 * bxx;
    const T n2yy = phi * uy * uy + R.p2 * byy;
    const T n2xy = phi * ux * uy + R.p2 * bxy;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int cx = ex(i), cy = ey(i);
        const T hxx = T(cx * cx) - r3, hyy = T(cy * cy) - r3;
        const T v = s0 + T(3) * (T(cx) * n1x + T(cy) * n1y) +
                    T(4.5) * (hxx * n2xx + hyy * n2yy + T(2 * cx * cy) * n2xy);
        out[i] = wgt<T>(i) * v;
    }
}

template <class T>
__device__ __forceinline__ bool wrap_cell(const RunDev<T>& R, int& xx, int& yy) {
    if (yy < 0 || yy >= R.ny) {
        if (R.ymode != XM_PERIODIC) return false;
        yy = ((yy % R.ny) + R.ny) % R.ny;
    }
    if (xx < 0 || xx >= R.nx) {
        if (R.xmode != XM_PERIODIC) return false;
        xx = ((xx % R.nx) + R.nx) % R.nx;
    }
    return true;
}

template <class T>
__device__ __forceinline__ unsigned node_bits(const RunDev<T>& R, int p) {
    return R.has_bits ? (unsigned)R.bits[p] : 0u;
}

// rho and u of one tile/ring cell (pull + hydrodynamic wall fill + moments).
template <class T>
__device__ __forceinline__ bool cell_macros(const RunDev<T>& R, const T* __restrict__ src, int cx,
                                            int cy, bool pull, T& rho, T& ux, T& uy) {
    if (!wrap_cell(R, cx, cy)) return false;
    const int p = cy * R.pitch + cx;
    const unsigned b = node_bits(R, p);
    if (b & BIT_SELF_SOLID) return false;
    Srcs s;
    node_srcs(R, cx, cy, b, pull, s);
    const int bi = (R.has_curved && (s.solid != 0u)) ? R.bidx[p] : -1;
    T f[9];
    load_hydro(R, src, cx, cy, s, bi, f);
    T Fx, Fy, drho;
    node_force(R, p, Fx, Fy);
    hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
    return true;
}

template <class T, int TY>
__global__ __launch_bounds__(64 * TY) void k_step(const RunDev<T>* __restrict__ runs,
                                                  const Item* __restrict__ items, int parity,
                                                  int first) {
    __shared__ T s_rho[TY + 2][66];
    __shared__ T s_ux[TY + 2][66];
    __shared__ T s_uy[TY + 2][66];
    const Item it = items[blockIdx.x];
    const RunDev<T>& R = runs[it.run];
    const T* __restrict__ src = R.pop[parity];
    T* __restrict__ dst = R.pop[parity ^ 1];
    const long long plane = R.plane;
    const bool pull = first == 0;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * 64 + lx;
    const int x0 = it.tx * 64, y0 = it.ty * TY;
    const int x = x0 + lx, y = y0 + ly;

    // ---- phase 1: own node (all 36 pulls, history, force) ----
    const bool in_dom = x < R.nx && y < R.ny;
    const int p = y * R.pitch + x;
    unsigned b = 0u;
    if (in_dom) b = node_bits(R, p);
    const bool active = in_dom && !(b & BIT_SELF_SOLID);
    Srcs s;
    T f[9], g[3][9];
    T Fx = T(0), Fy = T(0), hS[3] = {T(0), T(0), T(0)}, hux = T(0), huy = T(0);
    int bi = -1;
    if (active) {
        node_srcs(R, x, y, b, pull, s);
        if (R.has_curved && (b & 0x1FEu)) bi = R.bidx[p];
        load_hydro(R, src, x, y, s, bi, f);
#pragma unroll
        for (int k = 0; k < 3; ++k) load_cde(R, src, k, p, s, g[k]);
        node_force(R, p, Fx, Fy);
        if (!first) {
#pragma unroll
            for (int k = 0; k < 3; ++k) hS[k] = R.hist[k * plane + p];
            hux = R.hist[3 * plane + p];
            huy = R.hist[4 * plane + p];
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
    T drho = T(0), rho = T(1), ux = T(0), uy = T(0);
    if (active) {
        hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
        s_rho[ly + 1][lx + 1] = rho;
        s_ux[ly + 1][lx + 1] = ux;
        s_uy[ly + 1][lx + 1] = uy;
    } else {
        // out-of-domain tile cell: periodic image for the neighbours' differences
        T r, vx, vy;
        if (!in_dom && cell_macros(R, src, x, y, pull, r, vx, vy)) {
            s_rho[ly + 1][lx + 1] = r;
            s_ux[ly + 1][lx + 1] = vx;
            s_uy[ly + 1][lx + 1] = vy;
        }
    }
    __syncthreads();
    if (!active) return;

    // ---- phase 2 ----
    // neighbour values for the differences (reading of the paper's silent gradient):
    // LDS for fluid neighbours, wall formula at walls, inlet/outlet ghosts at open ends.
    const bool wxl = (b >> 1) & 1u, wxh = (b >> 3) & 1u, wyl = (b >> 2) & 1u, wyh = (b >> 4) & 1u;
    const int bq_row = bi;
    const T qxl = link_q(R, bq_row, 1), qxh = link_q(R, bq_row, 3);
    const T qyl = link_q(R, bq_row, 2), qyh = link_q(R, bq_row, 4);
    const bool open_l = R.xmode == XM_OPEN && x == 0;
    const bool open_h = R.xmode == XM_OPEN && x == R.nx - 1;
    T rl, uxl, uyl, rh, uxh, uyh;
    if (open_l) { rl = T(1); uxl = R.inlet[y]; uyl = T(0); }
    else if (!wxl) { rl = s_rho[ly + 1][lx]; uxl = s_ux[ly + 1][lx]; uyl = s_uy[ly + 1][lx]; }
    else { rl = T(0); uxl = T(0); uyl = T(0); }
    if (open_h) { rh = rho; uxh = ux; uyh = uy; }
    else if (!wxh) { rh = s_rho[ly + 1][lx + 2]; uxh = s_ux[ly + 1][lx + 2]; uyh = s_uy[ly + 1][lx + 2]; }
    else { rh = T(0); uxh = T(0); uyh = T(0); }
    T rd = T(0), uxd = T(0), uyd = T(0), ru = T(0), uxu = T(0), uyu = T(0);
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

    // conformation: phi_k (CNEBB at boundary nodes), Oldroyd-B stress and source
    T dphi[3];
    if (s.solid) {
#pragma unroll
        for (int k = 0; k < 3; ++k) cnebb(s.solid, k, ux, uy, g[k], dphi[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T acc = T(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) acc += g[k][i];
            dphi[k] = acc;
        }
    }
    const T axx = T(1) + dphi[0], axy = dphi[1], ayy = T(1) + dphi[2];
    const T txx = R.eta_over_lam * dphi[0], txy = R.eta_over_lam * dphi[1],
            tyy = R.eta_over_lam * dphi[2];
    T S[3];
    if (R.no_source) {
        S[0] = S[1] = S[2] = T(0);
    } else {
        const T d = Lxx + Lyy;
        S[0] = -R.inv_lam * dphi[0] + T(2) * (axx * Lxx + axy * Lyx) + axx * d;
        S[1] = -R.inv_lam * dphi[1] + axx * Lxy + axy * Lyy + axy * Lxx + ayy * Lyx + axy * d;
        S[2] = -R.inv_lam * dphi[2] + T(2) * (axy * Lxy + ayy * Lyy) + ayy * d;
    }
    if (first) {
        hS[0] = S[0]; hS[1] = S[1]; hS[2] = S[2];
        hux = ux; huy = uy;
    }

    T out[9];
    collide_hydro(R, f, drho, rho, ux, uy, Fx, Fy, txx, txy, tyy, Dx, Dy, out);
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[i * plane + p] = out[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T phi = phi0<T>(k) + dphi[k];
        collide_cde(R, g[k], dphi[k], phi, ux, uy, phi / rho, Fx, Fy, S[k], hS[k], hux, huy, out);
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[(9 + 9 * k + i) * plane + p] = out[i];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) R.hist[k * plane + p] = S[k];
    R.hist[3 * plane + p] = ux;
    R.hist[4 * plane + p] = uy;
}

// Equilibrium initial state into buffer 0; history cleared.
template <class T>
__global__ void k_init(const RunDev<T>* __restrict__ run, const T* rho0, const T* ux0,
                       const T* uy0, const T* a0, const T* a1, const T* a2) {
    const RunDev<T>& R = *run;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= R.nx || y >= R.ny) return;
    const int p = y * R.pitch + x;
    const int q = y * R.nx + x;
    const long long plane = R.plane;
    T* __restrict__ dst = R.pop[0];
    const bool solid = R.has_bits && (R.bits[p] & BIT_SELF_SOLID);
    const T r = rho0 ? rho0[q] : T(1);
    const T vx = ux0 ? ux0[q] : T(0), vy = uy0 ? uy0[q] : T(0);
    const T* a[3] = {a0, a1, a2};
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[i * plane + p] = solid ? T(0) : dfeq<T>(i, r - T(1), r, vx, vy);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T phi = a[k] ? a[k][q] : phi0<T>(k);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            dst[(9 + 9 * k + i) * plane + p] = solid ? T(0) : dgeq<T>(i, phi - phi0<T>(k), phi, vx, vy);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) R.hist[c * plane + p] = T(0);
}

// Macroscopic fields of node (x, y) at the current time; false for solid nodes.
template <class T>
__device__ __forceinline__ bool node_fields(const RunDev<T>& R, const T* __restrict__ src, int x,
                                            int y, bool pull, T& rho, T& ux, T& uy, T a[3]) {
    const int p = y * R.pitch + x;
    const unsigned b = node_bits(R, p);
    if (b & BIT_SELF_SOLID) return false;
    Srcs s;
    node_srcs(R, x, y, b, pull, s);
    const int bi = (R.has_curved && s.solid) ? R.bidx[p] : -1;
    T f[9];
    load_hydro(R, src, x, y, s, bi, f);
    T Fx, Fy, drho;
    node_force(R, p, Fx, Fy);
    hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T g[9];
        load_cde(R, src, k, p, s, g);
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) acc += g[i];
        a[k] = phi0<T>(k) + acc;  // phi_b at boundary nodes (CNEBB keeps it)
    }
    return true;
}

template <class T>
__global__ void k_read(const RunDev<T>* __restrict__ run, int parity, int first, T* rho_o,
                       T* ux_o, T* uy_o, T* axx_o, T* axy_o, T* ayy_o) {
    const RunDev<T>& R = *run;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= R.nx || y >= R.ny) return;
    const int q = y * R.nx + x;
    T r = T(0), vx = T(0), vy = T(0), a[3] = {T(0), T(0), T(0)};
    if (!node_fields(R, R.pop[parity], x, y, first == 0, r, vx, vy, a)) {
        r = T(0);
    }
    if (rho_o) rho_o[q] = r;
    if (ux_o) ux_o[q] = vx;
    if (uy_o) uy_o[q] = vy;
    if (axx_o) axx_o[q] = a[0];
    if (axy_o) axy_o[q] = a[1];
    if (ayy_o) ayy_o[q] = a[2];
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
template <class T>
__global__ __launch_bounds__(256) void k_monitor(const RunDev<T>* __restrict__ run, int parity,
                                                 int first, T* usnap, MonitorAcc* acc) {
    const RunDev<T>& R = *run;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    double m[4] = {0, 0, 0, 0}, res = 0, umax = 0, nf = 0, spd = 0;
    if (x < R.nx && y < R.ny) {
        T r, vx, vy, a[3];
        if (node_fields(R, R.pop[parity], x, y, first == 0, r, vx, vy, a)) {
            const int q = y * R.nx + x;
            const double dr = (double)r, dx = (double)vx, dy = (double)vy;
            const double ok = (isfinite(dr) && isfinite(dx) && isfinite(dy) &&
                               isfinite((double)a[0]) && isfinite((double)a[1]) &&
                               isfinite((double)a[2])) ? 1.0 : 0.0;
            if (ok != 0.0) {
                m[0] = dr; m[1] = (double)a[0]; m[2] = (double)a[1]; m[3] = (double)a[2];
                const double ex_ = dx - (double)usnap[q], ey_ = dy - (double)usnap[R.nx * R.ny + q];
                res = sqrt(ex_ * ex_ + ey_ * ey_);
                umax = sqrt(dx * dx + dy * dy);
                const double det = (double)a[0] * (double)a[2] - (double)a[1] * (double)a[1];
                spd = (det <= 0.0 || (double)a[0] + (double)a[2] <= 0.0) ? 1.0 : 0.0;
            } else {
                nf = 1.0;
            }
            usnap[q] = vx;
            usnap[R.nx * R.ny + q] = vy;
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

template <class T>
hipError_t launch_step(const RunDev<T>* runs_dev, const Item* items_dev, int nitems, int ty,
                       int parity, int first, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (ty) {
        case 1: hipLaunchKernelGGL((k_step<T, 1>), dim3(nitems), dim3(64, 1), 0, s, runs_dev, items_dev, parity, first); break;
        case 2: hipLaunchKernelGGL((k_step<T, 2>), dim3(nitems), dim3(64, 2), 0, s, runs_dev, items_dev, parity, first); break;
        case 4: hipLaunchKernelGGL((k_step<T, 4>), dim3(nitems), dim3(64, 4), 0, s, runs_dev, items_dev, parity, first); break;
        case 8: hipLaunchKernelGGL((k_step<T, 8>), dim3(nitems), dim3(64, 8), 0, s, runs_dev, items_dev, parity, first); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_init(const RunDev<T>& h, const RunDev<T>* d, const T* rho, const T* ux,
                       const T* uy, const T* axx, const T* axy, const T* ayy, hipStream_t s) {
    dim3 blk(64, 4), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_init<T>), grd, blk, 0, s, d, rho, ux, uy, axx, axy, ayy);
    return hipGetLastError();
}

template <class T>
hipError_t launch_read(const RunDev<T>& h, const RunDev<T>* d, int parity, int first, T* rho,
                       T* ux, T* uy, T* axx, T* axy, T* ayy, hipStream_t s) {
    dim3 blk(64, 4), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_read<T>), grd, blk, 0, s, d, parity, first, rho, ux, uy, axx, axy, ayy);
    return hipGetLastError();
}

template <class T>
hipError_t launch_monitor(const RunDev<T>& h, const RunDev<T>* d, int parity, int first,
                          T* usnap, MonitorAcc* acc, hipStream_t s) {
    dim3 blk(256), grd((h.nx + 63) / 64, (h.ny + 3) / 4);
    hipLaunchKernelGGL((k_monitor<T>), grd, blk, 0, s, d, parity, first, usnap, acc);
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

#define VLB_INSTANTIATE(T)                                                                   \
    template hipError_t launch_step<T>(const RunDev<T>*, const Item*, int, int, int, int,  \
                                       hipStream_t);                                       \
    template hipError_t launch_init<T>(const RunDev<T>&, const RunDev<T>*, const T*,       \
                                       const T*, const T*, const T*, const T*, const T*,  \
                                       hipStream_t);                                       \
    template hipError_t launch_read<T>(const RunDev<T>&, const RunDev<T>*, int, int, T*,   \
                                       T*, T*, T*, T*, T*, hipStream_t);                   \
    template hipError_t launch_monitor<T>(const RunDev<T>&, const RunDev<T>*, int, int,    \
                                          T*, MonitorAcc*, hipStream_t);
VLB_INSTANTIATE(float)
VLB_INSTANTIATE(double)

}  // namespace vlb
