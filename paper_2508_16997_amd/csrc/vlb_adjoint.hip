// vlb_adjoint.hip -- discrete adjoint of the coupled step on domains with periodic axes,
// half-way walls, solid nodes and curved (circle) walls.
//
// The reverse sweep of time step n maps the adjoint of the state after the step
// (post-streaming populations of all four lattices and the S/u history) to the adjoint
// of the state before it, and accumulates the parameter gradients.  Two launches:
//   k_adj_local   per node: recomputes the forward quantities of step n from the
//                 stored state exactly as the step kernel does (pulls, rho/u of a
//                 one-node ring in LDS, wall-aware differences, constitutive source),
//                 pulls the adjoint of its post-collision populations from x + e_i
//                 (transpose of the pull) or, on wall links, from the boundary rule's
//                 transpose (half-way or interpolated bounce-back for f, the copy into
//                 the CNEBB input for g), applies the transposed moment-form collisions,
//                 constitutive source and polymer stress, then the transpose of CNEBB
//                 at wall-adjacent nodes.  It writes the
//                 final conformation-lattice adjoints, the adjoint of the history
//                 input, per-node intermediates for the second pass, and adds its
//                 block's share of dL/dlambda and dL/deta_p.
//   k_adj_gather  per node: transpose of the finite differences (the velocity gradient
//                 and d(rho u^3) of the node and its four axis neighbours, each with the
//                 coefficients its own wall configuration gives them), then of the
//                 macroscopic moments (rho, u with the half-force shift): the final
//                 hydrodynamic adjoint populations; accumulates dL/dF in double.
// A seed kernel turns dL/du at the last step (or a target velocity, for the mean
// squared error over the fluid nodes) into the adjoint of the last state.
// Solid nodes carry zero adjoints: fluid nodes read the adjoints of the values their
// pulls took from solid slots at their own slot (the fill's transpose), never there.
// Arithmetic is double; adjoint planes use the storage type S of the forward state.
#include "vlb_device.h"

namespace vlb {
namespace {

// planes of the per-node scratch written by k_adj_local, read by k_adj_gather
enum {
    SC_MF = 0,                                     // 8: adjoint of the hydrodynamic moments
    SC_RHO = 8, SC_UX = 9, SC_UY = 10,             // local adjoints of rho, u
    SC_LXX = 11, SC_LXY = 12, SC_LYX = 13, SC_LYY = 14,  // adjoint of L[g][b] = d_g u_b
    SC_DX = 15, SC_DY = 16,                        // adjoint of d_x(rho ux^3), d_y(rho uy^3)
    SC_R = 17, SC_VX = 18, SC_VY = 19,             // forward rho, u
    SC_FX = 20, SC_FY = 21,                        // local adjoint of F
    SC_NPLANES = 22
};
static_assert(SC_NPLANES == 22, "scratch planes");

// Adjoint state planes: 0..8 hydrodynamic populations, 9..35 conformation lattices,
// 36..38 history S_xx, S_xy, S_yy, 39..40 history u_x, u_y.
constexpr int ADJ_HIST = 36;

__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Transpose of rebuild(): given the adjoints o of the nine outputs, the adjoints of
// (e0, M1, M2, M3).  Each output is w_i times a polynomial in e_i, so the transpose is
// a set of moments of w_i o_i.
struct RebuildAdj {
    T e0, m1x, m1y, m2xx, m2yy, m2xy, m3xxy, m3xyy;
};
__device__ __forceinline__ RebuildAdj rebuild_adj(const T o[9]) {
    T z[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) z[i] = wgt(i) * o[i];
    const Mom m = moments(z);
    RebuildAdj r;
    r.e0 = m.m0;
    r.m1x = 3.0 * m.mx;
    r.m1y = 3.0 * m.my;
    r.m2xx = 4.5 * (m.pxx - R3 * m.m0);
    r.m2yy = 4.5 * (m.pyy - R3 * m.m0);
    r.m2xy = 9.0 * m.pxy;
    r.m3xxy = 13.5 * (m.qxxy - R3 * m.my);
    r.m3xyy = 13.5 * (m.qxyy - R3 * m.mx);
    return r;
}

// Transpose of moments(): the adjoint of population i from the adjoints of the eight
// moments is the moment polynomial evaluated at e_i.
__device__ __forceinline__ void expand(const Mom& a, T v[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T cx = T(ex(i)), cy = T(ey(i));
        v[i] = a.m0 + cx * a.mx + cy * a.my + cx * cx * a.pxx + cy * cy * a.pyy + cx * cy * a.pxy +
               cx * cx * cy * a.qxxy + cx * cy * cy * a.qxyy;
    }
}

// Adjoint of collide_hydro() with the moments of f, rho, u, F, tau and (Dx, Dy) as
// independent inputs.
struct HydroAdj {
    Mom mf;
    T rho, ux, uy, Fx, Fy, txx, txy, tyy, Dx, Dy;
};
template <class S>
__device__ __forceinline__ void collide_hydro_adj(const RunDev<S>& R, T rho, T ux, T uy,
                                                  const T o[9], HydroAdj& a) {
    const RebuildAdj b = rebuild_adj(o);
    const T c1 = R.c1, c2 = R.c2, e1 = 1.0 - R.c1, e2 = 1.0 - R.c2;
    a.Fx = R.h1 * b.m1x;
    a.Fy = R.h1 * b.m1y;
    a.Dx = -R.h1 * b.m2xx;
    a.Dy = -R.h1 * b.m2yy;
    a.txx = -R.inv_ts1 * b.m2xx;
    a.tyy = -R.inv_ts1 * b.m2yy;
    a.txy = -R.inv_ts1 * b.m2xy;
    // raw moments of f: directly, and through the off-equilibrium moments a_n
    const T axx = c1 * b.m2xx, ayy = c1 * b.m2yy;
    const T axxy = c2 * b.m3xxy, axyy = c2 * b.m3xyy;
    a.mf.m0 = b.e0 - R3 * (axx + ayy);
    a.mf.mx = c1 * b.m1x - R3 * axyy;
    a.mf.my = c1 * b.m1y - R3 * axxy;
    a.mf.pxx = axx;
    a.mf.pyy = ayy;
    a.mf.pxy = c1 * b.m2xy;
    a.mf.qxxy = axxy;
    a.mf.qxyy = axyy;
    // equilibrium moments rho u, rho uu and rho uuu enter with weight 1 - c
    const T rux = e1 * b.m1x, ruy = e1 * b.m1y;
    const T ruxx = e1 * b.m2xx + e2 * uy * b.m3xxy;
    const T ruyy = e1 * b.m2yy + e2 * ux * b.m3xyy;
    const T ruxy = e1 * b.m2xy;
    a.rho = rux * ux + ruy * uy + ruxx * ux * ux + ruyy * uy * uy + ruxy * ux * uy;
    a.ux = rho * (rux + 2.0 * ruxx * ux + ruxy * uy) + e2 * rho * uy * uy * b.m3xyy;
    a.uy = rho * (ruy + 2.0 * ruyy * uy + ruxy * ux) + e2 * rho * ux * ux * b.m3xxy;
}

// Adjoint of collide_cde() with the moments of g, phi, u, fr = phi/rho, F, S, S_prev
// and u_prev as independent inputs.
struct CdeAdj {
    Mom mg;
    T phi, fr, ux, uy, Fx, Fy, S, Sp, uxp, uyp;
};
template <class S>
__device__ __forceinline__ void collide_cde_adj(const RunDev<S>& R, T phi, T ux, T uy, T fr, T Fx,
                                                T Fy, T Sk, T Sp, T uxp, T uyp, const T o[9],
                                                CdeAdj& a) {
    const RebuildAdj b = rebuild_adj(o);
    const T p1 = R.p1, p2 = R.p2, h2 = R.h2, q1 = 1.0 - R.p1, q2 = 1.0 - R.p2;
    // e0 = dphi + 1.5 S - 0.5 S_prev
    T dphi = b.e0;
    a.S = 1.5 * b.e0 + 1.5 * h2 * (ux * b.m1x + uy * b.m1y);
    a.Sp = -0.5 * b.e0 - 0.5 * h2 * (uxp * b.m1x + uyp * b.m1y);
    // N1 = phi u + p1 b_1 + h2 (F fr + 1.5 S u - 0.5 S_prev u_prev)
    T pux = q1 * b.m1x, puy = q1 * b.m1y;
    a.Fx = h2 * fr * b.m1x;
    a.Fy = h2 * fr * b.m1y;
    a.fr = h2 * (Fx * b.m1x + Fy * b.m1y);
    T aux = 1.5 * h2 * Sk * b.m1x, auy = 1.5 * h2 * Sk * b.m1y;
    a.uxp = -0.5 * h2 * Sp * b.m1x;
    a.uyp = -0.5 * h2 * Sp * b.m1y;
    // N2 = phi uu + p2 b_2 (xx, yy, xy)
    const T fux = phi * ux, fuy = phi * uy;
    pux += q2 * (ux * b.m2xx + uy * b.m2xy);
    puy += q2 * uy * b.m2yy;
    aux += q2 * fux * b.m2xx;
    auy += q2 * (fuy * b.m2yy + fux * b.m2xy);
    dphi -= p2 * R3 * (b.m2xx + b.m2yy);
    // phi u
    a.phi = pux * ux + puy * uy;
    a.ux = aux + pux * phi;
    a.uy = auy + puy * phi;
    a.mg.m0 = dphi;
    a.mg.mx = p1 * b.m1x;
    a.mg.my = p1 * b.m1y;
    a.mg.pxx = p2 * b.m2xx;
    a.mg.pyy = p2 * b.m2yy;
    a.mg.pxy = p2 * b.m2xy;
    a.mg.qxxy = 0.0;
    a.mg.qxyy = 0.0;
}

__device__ __forceinline__ int wrapm(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Transpose of cnebb() (conservative non-equilibrium bounce-back, Sec. 3.3) at a node with
// unknown set `solid` (bits 1..8): gr_i = E_i(s, u) + [opp(i) known] (g_opp(i) - E_opp(i)(s, u))
// for unknown i, gr_i = g_i for known i >= 1, gr_0 = s - sum_{i >= 1} gr_i, with
// s = sum_i g_i and E_i(s, u) = w_i [s + (phi0 + s) P_i(u)],
// P_i(u) = 3 e_i.u + 4.5 (e_i.u)^2 - 1.5 u.u.  Given the adjoints ga of gr, returns in ga
// the adjoints of the pulled g and adds the velocity adjoints to aux, auy.
__device__ __forceinline__ void cnebb_adj(unsigned solid, int k, T s, T ux, T uy, T ga[9], T& aux,
                                          T& auy) {
    const T phi = phi0(k) + s;
    T b[9], ag[9], as = ga[0];
#pragma unroll
    for (int i = 0; i < 9; ++i) ag[i] = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) b[i] = ga[i] - ga[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (!((solid >> i) & 1u)) {
            ag[i] += b[i];
            continue;
        }
        auto dE = [&](int j, T& ds, T& dx, T& dy) {
            const T cx = T(ex(j)), cy = T(ey(j));
            const T eu = cx * ux + cy * uy;
            ds = wgt(j) * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy));
            dx = wgt(j) * phi * (3.0 * cx + 9.0 * eu * cx - 3.0 * ux);
            dy = wgt(j) * phi * (3.0 * cy + 9.0 * eu * cy - 3.0 * uy);
        };
        T ds, dx, dy;
        dE(i, ds, dx, dy);
        const int o = opp(i);
        if (!((solid >> o) & 1u)) {
            T ds2, dx2, dy2;
            dE(o, ds2, dx2, dy2);
            ds -= ds2;
            dx -= dx2;
            dy -= dy2;
            ag[o] += b[i];
        }
        as += b[i] * ds;
        aux += b[i] * dx;
        auy += b[i] * dy;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) ga[i] = ag[i] + as;
}

// Coefficients of dgrad() along one axis of a node: the derivative is
// c[0] psi(low neighbour) + c[1] psi(node) + c[2] psi(high neighbour).
__device__ __forceinline__ void fd_coefs(bool lo_wall, T qlo, bool hi_wall, T qhi, T c[3]) {
    if (!lo_wall && !hi_wall) { c[0] = -0.5; c[1] = 0.0; c[2] = 0.5; }
    else if (lo_wall && !hi_wall) { c[0] = 0.0; c[1] = (1.0 - qlo) / qlo; c[2] = qlo / (1.0 + qlo); }
    else if (!lo_wall) { c[0] = -(qhi / (1.0 + qhi)); c[1] = -((1.0 - qhi) / qhi); c[2] = 0.0; }
    else { c[0] = 0.0; c[1] = (qhi - qlo) / (qlo * qhi); c[2] = 0.0; }
}
// Both axes of node slot p (x: low/high = directions 1/3, y: 2/4 as in the step kernel).
template <class S>
__device__ __forceinline__ void node_fd_coefs(const RunDev<S>& R, int p, unsigned b, T cx[3],
                                              T cy[3]) {
    T q1 = 0.5, q2 = 0.5, q3 = 0.5, q4 = 0.5;
    if (R.has_curved && (b & 0x1Eu)) {
        const int bi = R.bidx[p];
        q1 = link_q(R, bi, 1); q3 = link_q(R, bi, 3);
        q2 = link_q(R, bi, 2); q4 = link_q(R, bi, 4);
    }
    fd_coefs((b >> 1) & 1u, q1, (b >> 3) & 1u, q3, cx);
    fd_coefs((b >> 2) & 1u, q2, (b >> 4) & 1u, q4, cy);
}

// Slot of the neighbour x + e_i across periodic axes (unwrapped across walls, where
// the caller's geometry bits say it is not a fluid node).
template <class S>
__device__ __forceinline__ int nb_slot(const RunDev<S>& R, int x, int y, int dx, int dy) {
    int xx = x + dx, yy = y + dy;
    if (R.xmode == XM_PERIODIC) xx = wrapm(xx, R.nx);
    if (R.ymode == XM_PERIODIC) yy = wrapm(yy, R.ny);
    return node_index(R, xx, yy);
}

// Sum of one double over the block into slot[0] (+= when add, = otherwise).
template <int TY>
__device__ __forceinline__ void block_sum(T v, T* s_red, double* slot, bool add) {
    v = wave_sum(v);
    const int tid = threadIdx.y * 64 + threadIdx.x;
    if ((tid & 63) == 0) s_red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        T s = 0.0;
        for (int w = 0; w < TY; ++w) s += s_red[w];
        *slot = add ? *slot + s : s;
    }
    __syncthreads();
}

// Transpose of the finite differences and of the macroscopic moments at fluid node
// (x, y) (slot p, geometry bits b) from the per-node intermediates sc of the local pass:
// the final hydrodynamic adjoint populations v and this node's contributions to dL/dF.
template <class S, bool WALLS>
__device__ __forceinline__ void gather_at(const RunDev<S>& R, long long plane, const S* sc, int x,
                                          int y, unsigned p, unsigned b, T v[9], T& gFx, T& gFy) {
    auto rd = [&](int c, unsigned q) -> T { return ldu(sc + c * plane, q); };
    // The derivative along an axis at node n is c0(n) psi(n - e) + c1(n) psi(n) +
    // c2(n) psi(n + e) with coefficients set by n's own walls.  Node x enters its own
    // derivatives with c1(x), those of its fluid low neighbour with c2(low) and those of
    // its fluid high neighbour with c0(high).
    T cx[3], cy[3];
    node_fd_coefs(R, (int)p, b, cx, cy);
    T wLx[3] = {0.0, 0.0, 0.0}, wLy[3] = {0.0, 0.0, 0.0};  // a_Lxx/a_Lxy/a_Dx, a_Lyx/a_Lyy/a_Dy
    const int cxs[3] = {SC_LXX, SC_LXY, SC_DX}, cys[3] = {SC_LYX, SC_LYY, SC_DY};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        wLx[c] = cx[1] * rd(cxs[c], p);
        wLy[c] = cy[1] * rd(cys[c], p);
    }
    auto neighbour = [&](int bitdir, int dx, int dy, int slot_c, T* w, const int* chans) {
        if ((b >> bitdir) & 1u) return;  // not a fluid node
        const unsigned q = (unsigned)nb_slot(R, x, y, dx, dy);
        T c[3], cdum[3];
        const unsigned bn = WALLS ? node_bits(R, (int)q) : 0u;
        if (dx != 0) node_fd_coefs(R, (int)q, bn, c, cdum);
        else node_fd_coefs(R, (int)q, bn, cdum, c);
#pragma unroll
        for (int k = 0; k < 3; ++k) w[k] += c[slot_c] * rd(chans[k], q);
    };
    neighbour(1, -1, 0, 2, wLx, cxs);  // low x neighbour: x is its high neighbour
    neighbour(3, 1, 0, 0, wLx, cxs);
    neighbour(2, 0, -1, 2, wLy, cys);
    neighbour(4, 0, 1, 0, wLy, cys);

    const T rho = rd(SC_R, p), ux = rd(SC_VX, p), uy = rd(SC_VY, p);
    T a_rho = rd(SC_RHO, p), a_ux = rd(SC_UX, p), a_uy = rd(SC_UY, p);
    a_ux += wLx[0] + wLy[0];
    a_uy += wLx[1] + wLy[1];
    const T a_px = wLx[2], a_py = wLy[2];  // adjoints of rho ux^3, rho uy^3
    a_rho += a_px * ux * ux * ux + a_py * uy * uy * uy;
    a_ux += 3.0 * a_px * rho * ux * ux;
    a_uy += 3.0 * a_py * rho * uy * uy;
    // rho = 1 + sum f, u = (j + F/2) / rho
    const T inv = 1.0 / rho;
    Mom m;
    m.m0 = rd(SC_MF + 0, p) + a_rho - (ux * a_ux + uy * a_uy) * inv;
    m.mx = rd(SC_MF + 1, p) + a_ux * inv;
    m.my = rd(SC_MF + 2, p) + a_uy * inv;
    m.pxx = rd(SC_MF + 3, p);
    m.pyy = rd(SC_MF + 4, p);
    m.pxy = rd(SC_MF + 5, p);
    m.qxxy = rd(SC_MF + 6, p);
    m.qxyy = rd(SC_MF + 7, p);
    expand(m, v);
    gFx = rd(SC_FX, p) + 0.5 * a_ux * inv;
    gFy = rd(SC_FY, p) + 0.5 * a_uy * inv;
}

// WALLS = false compiles the periodic form (no geometry bits: every wall branch folds
// away and the kernel keeps the register budget of three waves per SIMD).
// FUSED: the hydrodynamic adjoints of the state after this step -- the gather of the
// later step, from its intermediates scr_in -- are formed here for the tile and its
// one-node ring into LDS (rounded to the storage type, as the separate gather stores
// them) instead of being read from ain, and this tile's dL/dF contributions of that
// gather are added; ain then supplies the conformation and history adjoints only.
// Not FUSED (the first reverse step): all of them come from ain.  Intermediates of this
// step go to scr_out (a different buffer: other tiles' rings still read scr_in).
template <class S, int TY, bool WALLS, bool FUSED>
__global__ __launch_bounds__(64 * TY, 2) void k_adj_local(const RunDev<S>* __restrict__ run,
                                                       const AdjDev<S>* __restrict__ adj,
                                                       const Item* __restrict__ items, int first,
                                                       const S* __restrict__ ain,
                                                       S* __restrict__ aout,
                                                       const S* __restrict__ scr_in,
                                                       S* __restrict__ scr_out) {
    __shared__ T s_rho[TY + 2][66];
    __shared__ T s_ux[TY + 2][66];
    __shared__ T s_uy[TY + 2][66];
    __shared__ T s_red[TY];
    constexpr int AF = FUSED ? 9 : 1, AFY = FUSED ? TY + 2 : 1, AFX = FUSED ? 66 : 1;
    __shared__ S s_af[AF][AFY][AFX];
    const Item it = items[blockIdx.x];
    const RunDev<S>& R = *run;
    const AdjDev<S>& A = *adj;
    const S* src = R.pop[0];
    const long long plane = R.plane;
    const bool pull = first == 0;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * 64 + lx;
    const int x0 = it.tx * 64, y0 = it.ty * TY;
    const int x = x0 + lx, y = y0 + ly;
    const bool in_dom = x < R.nx && y < R.ny;
    const int p = node_index(R, x, y);
    const unsigned b = (WALLS && in_dom) ? node_bits(R, p) : 0u;
    const bool active = in_dom && !(b & BIT_SELF_SOLID);

    // ---- forward front end of step n (as in the step kernel) ----
    S f[9], g[3][9];
    T Fx = 0.0, Fy = 0.0, hS[3] = {0.0, 0.0, 0.0}, hux = 0.0, huy = 0.0;
    if (FUSED) {
        // gather of the later step over the tile and its ring (wrapped on every axis, as
        // the pulls' neighbours are; cells no fluid node of the tile reads are harmless
        // extra work); the tile's own nodes add that gather's dL/dF, each node once over
        // the grid, in the order of the reverse steps as the separate gather did
        for (int r = tid; r < (TY + 2) * 66; r += 64 * TY) {
            const int lcy = r / 66, lcx = r - lcy * 66;
            const int cx = x0 - 1 + lcx, cy = y0 - 1 + lcy;
            const int wx = ((cx % R.nx) + R.nx) % R.nx, wy = ((cy % R.ny) + R.ny) % R.ny;
            const unsigned q = (unsigned)node_index(R, wx, wy);
            const unsigned bq = WALLS ? node_bits(R, (int)q) : 0u;
            if (bq & BIT_SELF_SOLID) continue;
            T v[9], fx, fy;
            gather_at<S, WALLS>(R, plane, scr_in, wx, wy, q, bq, v, fx, fy);
#pragma unroll
            for (int i = 0; i < 9; ++i) s_af[i][lcy][lcx] = (S)v[i];
            if (lcx >= 1 && lcx <= 64 && lcy >= 1 && lcy <= TY && cx < R.nx && cy < R.ny) {
                A.gF[q] += fx;
                A.gF[plane + q] += fy;
            }
        }
    }
    if (active) {
        pull36(R, src, p, pull, f, g);
        node_force(R, p, Fx, Fy);
        if (pull) hist_ld(R.hist, plane, (unsigned)p, hS, hux, huy);
    }
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
        T rr, vx, vy;
        if (cell_macros(R, src, x, y, pull, rr, vx, vy)) {
            s_rho[ly + 1][lx + 1] = rr;
            s_ux[ly + 1][lx + 1] = vx;
            s_uy[ly + 1][lx + 1] = vy;
        }
    }
    __syncthreads();

    T glam = 0.0, geta = 0.0;
    if (in_dom && !active) {
        // solid node: nothing flows through it
        for (int c = 0; c < 41; ++c) stu(aout + c * plane, (unsigned)p, 0.0);
        for (int c = 0; c < SC_NPLANES; ++c) stu(scr_out + c * plane, (unsigned)p, 0.0);
    }
    if (active) {
        // velocity gradient by the step kernel's differences (wall-aware at fraction q)
        const bool wxl = (b >> 1) & 1u, wxh = (b >> 3) & 1u, wyl = (b >> 2) & 1u, wyh = (b >> 4) & 1u;
        const T uxl = wxl ? 0.0 : s_ux[ly + 1][lx], uyl = wxl ? 0.0 : s_uy[ly + 1][lx];
        const T uxh = wxh ? 0.0 : s_ux[ly + 1][lx + 2], uyh = wxh ? 0.0 : s_uy[ly + 1][lx + 2];
        const T uxd = wyl ? 0.0 : s_ux[ly][lx + 1], uyd = wyl ? 0.0 : s_uy[ly][lx + 1];
        const T uxu = wyh ? 0.0 : s_ux[ly + 2][lx + 1], uyu = wyh ? 0.0 : s_uy[ly + 2][lx + 1];
        T qq[5] = {0.5, 0.5, 0.5, 0.5, 0.5};
        if (R.has_curved && (b & 0x1Eu)) {
            const int bi = R.bidx[p];
            for (int i = 1; i <= 4; ++i) qq[i] = link_q(R, bi, i);
        }
        const T Lxx = dgrad(wxl, qq[1], uxl, ux, wxh, qq[3], uxh);
        const T Lxy = dgrad(wxl, qq[1], uyl, uy, wxh, qq[3], uyh);
        const T Lyx = dgrad(wyl, qq[2], uxd, ux, wyh, qq[4], uxu);
        const T Lyy = dgrad(wyl, qq[2], uyd, uy, wyh, qq[4], uyu);

        Mom gm[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) gm[k] = moments(g[k]);
        const T d0 = gm[0].m0, d1 = gm[1].m0, d2 = gm[2].m0;
        const T axx = 1.0 + d0, axy = d1, ayy = 1.0 + d2;
        T rf[3] = {d0, d1, d2}, sf[3] = {d0, d1, d2};
        if (R.model != MODEL_OLDROYD_B) closure(R.model, R.mpar, d0, d1, d2, rf, sf);
        T Sc[3] = {0.0, 0.0, 0.0};
        if (!R.no_source) {
            const T d = Lxx + Lyy;
            Sc[0] = -R.inv_lam * rf[0] + 2.0 * (axx * Lxx + axy * Lyx) + axx * d;
            Sc[1] = -R.inv_lam * rf[1] + axx * Lxy + axy * Lyy + axy * Lxx + ayy * Lyx + axy * d;
            Sc[2] = -R.inv_lam * rf[2] + 2.0 * (axy * Lxy + ayy * Lyy) + ayy * d;
        }
        if (!pull) {
            hS[0] = Sc[0]; hS[1] = Sc[1]; hS[2] = Sc[2];
            hux = ux; huy = uy;
        }

        // Adjoint of the post-collision population of direction i: where it streams --
        // the neighbour x + e_i (across periodic axes) -- or, when that neighbour is
        // solid, the boundary rule of this node's pull in direction opp(i) that used it
        // (the transpose of k_fill).  Interpolated bounce-back on a curved link of
        // fraction q (pull direction d, o = opp(d), far = x + e_d):
        //   q < 1/2: f_d(x) = 2q f_o(x) + (1 - 2q) f_o(far)   (half-way if far is solid)
        //   q >= 1/2: f_d(x) = f_o(x) / 2q + (2q - 1) / 2q f_d(x)
        // so f_i(x) also feeds the pull of x in direction i (second branch) and, as
        // f_o(far), the pull of the neighbour x + e_i in direction opp(i) (first branch).
        // The conformation lattices copy f_o(x) into the CNEBB input of direction d.
        // (wrapped on every axis: a neighbour across a wall axis is never fluid, so its
        // slot is never used)
        const int xl = wrapm(x - 1, R.nx), xh = wrapm(x + 1, R.nx);
        const int yl = wrapm(y - 1, R.ny), yh = wrapm(y + 1, R.ny);
        const int row[3] = {R.off0 + yl * R.pitch, R.off0 + y * R.pitch, R.off0 + yh * R.pitch};
        const int col[3] = {xl, x, xh};
        auto nb = [&](int i) -> unsigned { return (unsigned)(row[1 + ey(i)] + col[1 + ex(i)]); };
        auto lq = [&](unsigned bits, int slot, int i) -> T {
            return (WALLS && R.has_curved && ((bits >> i) & 1u)) ? link_q(R, R.bidx[slot], i)
                                                                 : 0.5;
        };
        auto solid_nb = [&](int i) -> bool { return (b >> opp(i)) & 1u; };

        // hydrodynamic adjoint of direction c at the node (dx, dy) from this one (slot)
        auto afh = [&](int c, int dx, int dy, unsigned slot) -> T {
            if constexpr (FUSED) return (T)s_af[c][ly + 1 + dy][lx + 1 + dx];
            else return ldu(ain + c * plane, slot);
        };
        T o[9];
        o[0] = afh(0, 0, 0, (unsigned)p);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int d = opp(i);
            T v;
            if (!solid_nb(i)) {
                const unsigned q_ = nb(i);
                v = afh(i, ex(i), ey(i), q_);
                if (WALLS && R.has_curved) {
                    // (first branch at the neighbour) x + e_i pulls d from x + 2 e_i
                    const unsigned bn = node_bits(R, (int)q_);
                    if ((bn >> d) & 1u) {
                        const T qn = lq(bn, (int)q_, d);
                        if (qn < 0.5) v += (1.0 - 2.0 * qn) * afh(d, ex(i), ey(i), q_);
                    }
                }
            } else {
                const T q = lq(b, p, d);
                T alpha;
                if (q < 0.5) alpha = ((b >> i) & 1u) ? 1.0 : 2.0 * q;  // far = x - e_i
                else alpha = 1.0 / (2.0 * q);
                v = alpha * afh(d, 0, 0, (unsigned)p);
            }
            if ((b >> i) & 1u) {
                // (second branch) this node pulls i from x - e_i solid with q > 1/2
                const T q = lq(b, p, i);
                if (q > 0.5) v += (2.0 * q - 1.0) / (2.0 * q) * afh(i, 0, 0, (unsigned)p);
            }
            o[i] = v;
        }
        HydroAdj ha;
        collide_hydro_adj(R, rho, ux, uy, o, ha);
        T a_rho = ha.rho, a_ux = ha.ux, a_uy = ha.uy, a_Fx = ha.Fx, a_Fy = ha.Fy;
        // this step's S and u became the next step's history
        T a_S[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) a_S[k] = ldu(ain + (ADJ_HIST + k) * plane, (unsigned)p);
        a_ux += ldu(ain + (ADJ_HIST + 3) * plane, (unsigned)p);
        a_uy += ldu(ain + (ADJ_HIST + 4) * plane, (unsigned)p);

        const T inv_rho = 1.0 / rho;
        T a_Sp[3], a_uxp = 0.0, a_uyp = 0.0, a_d[3];
        Mom a_mg[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[0] = ldu(ain + (9 + 9 * k) * plane, (unsigned)p);
#pragma unroll
            for (int i = 1; i < 9; ++i)
                o[i] = solid_nb(i) ? ldu(ain + (9 + 9 * k + opp(i)) * plane, (unsigned)p)
                                   : ldu(ain + (9 + 9 * k + i) * plane, nb(i));
            const T phi = phi0(k) + gm[k].m0;
            const T fr = phi * inv_rho;
            CdeAdj ca;
            collide_cde_adj(R, phi, ux, uy, fr, Fx, Fy, Sc[k], hS[k], hux, huy, o, ca);
            a_mg[k] = ca.mg;
            a_d[k] = ca.phi + ca.fr * inv_rho;      // phi = phi0 + d_k, fr = phi / rho
            a_rho -= ca.fr * phi * inv_rho * inv_rho;
            a_S[k] += ca.S;
            a_Sp[k] = ca.Sp;
            a_ux += ca.ux;
            a_uy += ca.uy;
            a_uxp += ca.uxp;
            a_uyp += ca.uyp;
            a_Fx += ca.Fx;
            a_Fy += ca.Fy;
        }
        if (!pull) {  // first step: S_prev = S, u_prev = u
#pragma unroll
            for (int k = 0; k < 3; ++k) { a_S[k] += a_Sp[k]; a_Sp[k] = 0.0; }
            a_ux += a_uxp;
            a_uy += a_uyp;
            a_uxp = 0.0;
            a_uyp = 0.0;
        }

        // constitutive source S(A, L, lambda) = -F_r(A)/lambda + upper-convected terms,
        // polymer stress tau = (eta_p / lambda) F_s(A)
        T a_Lxx = 0.0, a_Lxy = 0.0, a_Lyx = 0.0, a_Lyy = 0.0;
        T wr[3] = {0.0, 0.0, 0.0};
        if (!R.no_source) {
            const T d = Lxx + Lyy;
            a_d[0] += a_S[0] * (2.0 * Lxx + d) + a_S[1] * Lxy;
            a_d[1] += a_S[0] * (2.0 * Lyx) + a_S[1] * (Lyy + Lxx + d) + a_S[2] * (2.0 * Lxy);
            a_d[2] += a_S[1] * Lyx + a_S[2] * (2.0 * Lyy + d);
            a_Lxx = 3.0 * axx * a_S[0] + 2.0 * axy * a_S[1] + ayy * a_S[2];
            a_Lyy = axx * a_S[0] + 2.0 * axy * a_S[1] + 3.0 * ayy * a_S[2];
            a_Lxy = axx * a_S[1] + 2.0 * axy * a_S[2];
            a_Lyx = 2.0 * axy * a_S[0] + ayy * a_S[1];
            glam += R.inv_lam * R.inv_lam * (rf[0] * a_S[0] + rf[1] * a_S[1] + rf[2] * a_S[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k) wr[k] = -R.inv_lam * a_S[k];
        }
        const T td = sf[0] * ha.txx + sf[1] * ha.txy + sf[2] * ha.tyy;
        const T ws[3] = {R.eta_over_lam * ha.txx, R.eta_over_lam * ha.txy, R.eta_over_lam * ha.tyy};
        T a_b[3];
        closure_adj(R.model, R.mpar, d0, d1, d2, wr, ws, a_b);
#pragma unroll
        for (int k = 0; k < 3; ++k) a_d[k] += a_b[k];
        geta += R.inv_lam * td;
        glam -= R.eta_over_lam * R.inv_lam * td;

        // final adjoints of the conformation populations and of the history input; at a
        // wall-adjacent node the moments other than the zeroth were taken of the CNEBB
        // reconstruction, the zeroth of the pulled populations (CNEBB keeps it)
        const unsigned solid = pull ? (b & 0x1FEu) : 0u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T v[9];
            if (solid) {
                const T a0 = a_mg[k].m0 + a_d[k];
                a_mg[k].m0 = 0.0;
                expand(a_mg[k], v);
                T au_x = 0.0, au_y = 0.0;
                cnebb_adj(solid, k, gm[k].m0, ux, uy, v, au_x, au_y);
#pragma unroll
                for (int i = 0; i < 9; ++i) v[i] += a0;
                a_ux += au_x;
                a_uy += au_y;
            } else {
                a_mg[k].m0 += a_d[k];
                expand(a_mg[k], v);
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) stu(aout + (9 + 9 * k + i) * plane, (unsigned)p, v[i]);
            stu(aout + (ADJ_HIST + k) * plane, (unsigned)p, a_Sp[k]);
        }
        stu(aout + (ADJ_HIST + 3) * plane, (unsigned)p, a_uxp);
        stu(aout + (ADJ_HIST + 4) * plane, (unsigned)p, a_uyp);

        S* sc = scr_out;
        const T mfv[8] = {ha.mf.m0, ha.mf.mx, ha.mf.my, ha.mf.pxx, ha.mf.pyy, ha.mf.pxy,
                          ha.mf.qxxy, ha.mf.qxyy};
#pragma unroll
        for (int c = 0; c < 8; ++c) stu(sc + (SC_MF + c) * plane, (unsigned)p, mfv[c]);
        stu(sc + SC_RHO * plane, (unsigned)p, a_rho);
        stu(sc + SC_UX * plane, (unsigned)p, a_ux);
        stu(sc + SC_UY * plane, (unsigned)p, a_uy);
        stu(sc + SC_LXX * plane, (unsigned)p, a_Lxx);
        stu(sc + SC_LXY * plane, (unsigned)p, a_Lxy);
        stu(sc + SC_LYX * plane, (unsigned)p, a_Lyx);
        stu(sc + SC_LYY * plane, (unsigned)p, a_Lyy);
        stu(sc + SC_DX * plane, (unsigned)p, ha.Dx);
        stu(sc + SC_DY * plane, (unsigned)p, ha.Dy);
        stu(sc + SC_R * plane, (unsigned)p, rho);
        stu(sc + SC_VX * plane, (unsigned)p, ux);
        stu(sc + SC_VY * plane, (unsigned)p, uy);
        stu(sc + SC_FX * plane, (unsigned)p, a_Fx);
        stu(sc + SC_FY * plane, (unsigned)p, a_Fy);
    }
    block_sum<TY>(glam, s_red, A.part + 2 * blockIdx.x, true);
    block_sum<TY>(geta, s_red, A.part + 2 * blockIdx.x + 1, true);
}

// The gather as a launch of its own: after the last reverse step (step 0), whose
// hydrodynamic adjoints no later step takes into its own launch.
template <class S, int TY, bool WALLS>
__global__ __launch_bounds__(64 * TY) void k_adj_gather(const RunDev<S>* __restrict__ run,
                                                        const AdjDev<S>* __restrict__ adj,
                                                        const Item* __restrict__ items,
                                                        const S* __restrict__ scr,
                                                        S* __restrict__ aout) {
    const Item it = items[blockIdx.x];
    const RunDev<S>& R = *run;
    const AdjDev<S>& A = *adj;
    const int x = it.tx * 64 + (int)threadIdx.x, y = it.ty * TY + (int)threadIdx.y;
    if (x >= A.nx || y >= A.ny) return;
    const long long plane = A.plane;
    const unsigned p = (unsigned)node_index(R, x, y);
    const unsigned b = WALLS ? node_bits(R, (int)p) : 0u;
    if (b & BIT_SELF_SOLID) return;
    T v[9], gFx, gFy;
    gather_at<S, WALLS>(R, plane, scr, x, y, p, b, v, gFx, gFy);
#pragma unroll
    for (int i = 0; i < 9; ++i) stu(aout + i * plane, p, v[i]);
    double* gF = A.gF;
    gF[p] += gFx;
    gF[plane + p] += gFy;
}

// Adjoint of the state after the last step from dL/du there (u read out with the
// half-force shift), or from a target velocity for L = (1/2N) sum |u - u*|^2.
template <class S, int TY>
__global__ __launch_bounds__(64 * TY) void k_adj_seed(const RunDev<S>* __restrict__ run,
                                                      const AdjDev<S>* __restrict__ adj,
                                                      const Item* __restrict__ items,
                                                      const S* __restrict__ src, int pull,
                                                      S* __restrict__ aout) {
    __shared__ T s_red[TY];
    const Item it = items[blockIdx.x];
    const RunDev<S>& R = *run;
    const AdjDev<S>& A = *adj;
    const long long plane = R.plane;
    const int x = it.tx * 64 + (int)threadIdx.x, y = it.ty * TY + (int)threadIdx.y;
    T loss = 0.0;
    if (x < R.nx && y < R.ny && (node_bits(R, node_index(R, x, y)) & BIT_SELF_SOLID)) {
        const int p = node_index(R, x, y);
        for (int c = 0; c < 41; ++c) stu(aout + c * plane, (unsigned)p, 0.0);
        A.gF[p] = 0.0;
        A.gF[plane + p] = 0.0;
    } else if (x < R.nx && y < R.ny) {
        const int p = node_index(R, x, y);
        S f[9];
        pull9(R, src, 0, p, pull != 0, f);
        T Fx, Fy, drho, rho, ux, uy;
        node_force(R, p, Fx, Fy);
        hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
        const int q = y * R.nx + x;
        T gx = T(A.seed_x[q]), gy = T(A.seed_y[q]);
        if (A.seed_is_target) {
            const T dx = ux - gx, dy = uy - gy;
            loss = 0.5 * (dx * dx + dy * dy) * A.inv_nfluid;
            gx = dx * A.inv_nfluid;
            gy = dy * A.inv_nfluid;
        }
        const T inv = 1.0 / rho;
        Mom m{};
        m.m0 = -(ux * gx + uy * gy) * inv;
        m.mx = gx * inv;
        m.my = gy * inv;
        T v[9];
        expand(m, v);
#pragma unroll
        for (int i = 0; i < 9; ++i) stu(aout + i * plane, (unsigned)p, v[i]);
        for (int c = 9; c < 41; ++c) stu(aout + c * plane, (unsigned)p, 0.0);
        A.gF[p] = 0.5 * gx * inv;
        A.gF[plane + p] = 0.5 * gy * inv;
    }
    block_sum<TY>(loss, s_red, A.lossp + blockIdx.x, false);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        A.part[2 * blockIdx.x] = 0.0;
        A.part[2 * blockIdx.x + 1] = 0.0;
    }
}

}  // namespace

template <class S>
hipError_t launch_adj_seed(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                           int nitems, int ty, const S* src, int pull, S* aout, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (ty) {
        case 1: hipLaunchKernelGGL((k_adj_seed<S, 1>), dim3(nitems), dim3(64, 1), 0, s, run_dev, adj_dev, items, src, pull, aout); break;
        case 2: hipLaunchKernelGGL((k_adj_seed<S, 2>), dim3(nitems), dim3(64, 2), 0, s, run_dev, adj_dev, items, src, pull, aout); break;
        case 4: hipLaunchKernelGGL((k_adj_seed<S, 4>), dim3(nitems), dim3(64, 4), 0, s, run_dev, adj_dev, items, src, pull, aout); break;
        case 8: hipLaunchKernelGGL((k_adj_seed<S, 8>), dim3(nitems), dim3(64, 8), 0, s, run_dev, adj_dev, items, src, pull, aout); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S, bool WALLS, bool FUSED>
hipError_t launch_adj_local_w(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                              int nitems, int ty, int first, const S* ain, S* aout,
                              const S* scr_in, S* scr_out, hipStream_t s) {
    switch (ty) {
        case 1: hipLaunchKernelGGL((k_adj_local<S, 1, WALLS, FUSED>), dim3(nitems), dim3(64, 1), 0, s, run_dev, adj_dev, items, first, ain, aout, scr_in, scr_out); break;
        case 2: hipLaunchKernelGGL((k_adj_local<S, 2, WALLS, FUSED>), dim3(nitems), dim3(64, 2), 0, s, run_dev, adj_dev, items, first, ain, aout, scr_in, scr_out); break;
        case 4: hipLaunchKernelGGL((k_adj_local<S, 4, WALLS, FUSED>), dim3(nitems), dim3(64, 4), 0, s, run_dev, adj_dev, items, first, ain, aout, scr_in, scr_out); break;
        case 8: hipLaunchKernelGGL((k_adj_local<S, 8, WALLS, FUSED>), dim3(nitems), dim3(64, 8), 0, s, run_dev, adj_dev, items, first, ain, aout, scr_in, scr_out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S, bool WALLS>
hipError_t launch_adj_gather_w(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                               int nitems, int ty, const S* scr, S* aout, hipStream_t s) {
    switch (ty) {
        case 1: hipLaunchKernelGGL((k_adj_gather<S, 1, WALLS>), dim3(nitems), dim3(64, 1), 0, s, run_dev, adj_dev, items, scr, aout); break;
        case 2: hipLaunchKernelGGL((k_adj_gather<S, 2, WALLS>), dim3(nitems), dim3(64, 2), 0, s, run_dev, adj_dev, items, scr, aout); break;
        case 4: hipLaunchKernelGGL((k_adj_gather<S, 4, WALLS>), dim3(nitems), dim3(64, 4), 0, s, run_dev, adj_dev, items, scr, aout); break;
        case 8: hipLaunchKernelGGL((k_adj_gather<S, 8, WALLS>), dim3(nitems), dim3(64, 8), 0, s, run_dev, adj_dev, items, scr, aout); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class S>
hipError_t launch_adj_step(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                           int nitems, int ty, int first, int walls, int fused, const S* ain,
                           S* aout, const S* scr_in, S* scr_out, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (walls)
        return fused ? launch_adj_local_w<S, true, true>(run_dev, adj_dev, items, nitems, ty, first, ain, aout, scr_in, scr_out, s)
                     : launch_adj_local_w<S, true, false>(run_dev, adj_dev, items, nitems, ty, first, ain, aout, scr_in, scr_out, s);
    return fused ? launch_adj_local_w<S, false, true>(run_dev, adj_dev, items, nitems, ty, first, ain, aout, scr_in, scr_out, s)
                 : launch_adj_local_w<S, false, false>(run_dev, adj_dev, items, nitems, ty, first, ain, aout, scr_in, scr_out, s);
}

template <class S>
hipError_t launch_adj_gather(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                             int nitems, int ty, int walls, const S* scr, S* aout, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    return walls ? launch_adj_gather_w<S, true>(run_dev, adj_dev, items, nitems, ty, scr, aout, s)
                 : launch_adj_gather_w<S, false>(run_dev, adj_dev, items, nitems, ty, scr, aout, s);
}

template hipError_t launch_adj_seed<float>(const RunDev<float>*, const AdjDev<float>*, const Item*, int, int, const float*, int, float*, hipStream_t);
template hipError_t launch_adj_seed<double>(const RunDev<double>*, const AdjDev<double>*, const Item*, int, int, const double*, int, double*, hipStream_t);
template hipError_t launch_adj_step<float>(const RunDev<float>*, const AdjDev<float>*, const Item*, int, int, int, int, int, const float*, float*, const float*, float*, hipStream_t);
template hipError_t launch_adj_step<double>(const RunDev<double>*, const AdjDev<double>*, const Item*, int, int, int, int, int, const double*, double*, const double*, double*, hipStream_t);
template hipError_t launch_adj_gather<float>(const RunDev<float>*, const AdjDev<float>*, const Item*, int, int, int, const float*, float*, hipStream_t);
template hipError_t launch_adj_gather<double>(const RunDev<double>*, const AdjDev<double>*, const Item*, int, int, int, const double*, double*, hipStream_t);

}  // namespace vlb
