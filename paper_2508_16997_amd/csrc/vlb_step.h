// vlb_step.h -- one coupled lattice Boltzmann step of a 64 x TY tile: the device code
// shared by the per-step kernel (k_step, vlb_kernels.hip) and the persistent batch kernel
// (k_batch, vlb_batch.hip), so both round identically.
//
// Every lane pulls its node's 36 post-collision populations from the neighbours' slots
// with one branch-free global load each (structure-of-arrays planes, x fastest, 64 lanes
// read contiguous rows).  Slots that do not hold a fluid node -- ghost rows/columns
// around the domain and solid nodes -- hold exactly the value the boundary rule gives for
// that link: periodic images and open-end ghosts are stored a second time by the edge
// lanes of the step, every other boundary link by the fill list (apply_fill_op).  rho
// and u of the tile and of a one-node ring around it go to LDS; then the velocity
// gradient and d(rho u^3) by finite differences, CNEBB at wall-adjacent nodes, the
// constitutive source, the hydrodynamic and three convection-diffusion collisions in
// moment form, and 36 + 5 coalesced stores.
// Storage is float or double (template S); populations are kept as deviations from
// the rest state (f_i - w_i, g_i - w_i phi0 with phi0 = 1, 0, 1).  All arithmetic is
// double precision: on CDNA the vector FP64 rate equals the unpacked FP32 rate, and
// single-precision arithmetic lets rounding drift accumulate over many steps.
// The collision is the paper's regularized TRT operator rewritten in Hermite-moment
// space (algebraically identical to the per-direction form).
#pragma once

#include "vlb_device.h"

// Register budget of the step kernel: W waves per SIMD for single-precision storage
// (124-126 VGPRs, no spills, at either W); double precision at its natural allocation
// (170 VGPRs, two waves, no spills; a budget of three waves spills 20 bytes per lane).
template <class S, int TY, int W>
struct StepBounds {
    static constexpr int threads = 64 * TY;
    static constexpr int min_waves_per_eu = sizeof(S) == 4 ? W : 1;
    // the persistent batch kernel loops over tiles and keeps a few more values live:
    // three waves per SIMD for single precision, two for double, without spills
    static constexpr int batch_waves_per_eu = sizeof(S) == 4 ? 3 : 2;
};

namespace vlb {
namespace {

// Ghost slots that the inlet (outlet) links of row y pull from: direction i with
// e_x = +1 (-1) is pulled by node (x, y + e_y) from (gx, y), gx = -1 (nx); at a periodic
// y edge the puller wraps and the slot is the corner ghost it pulls from.  Calls
// fn(i, slot) for each.
template <class S, class F>
__device__ __forceinline__ void open_end_slots(const RunDev<S>& R, int y, bool in, F fn) {
    const int gx = in ? -1 : R.nx;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (ex(i) != (in ? 1 : -1)) continue;
        const int yp = y + ey(i);
        int gy = y;
        if (yp < 0 || yp >= R.ny) {
            if (R.ymode != XM_PERIODIC) continue;  // beyond a wall: nobody pulls it
            gy = (yp < 0 ? yp + R.ny : yp - R.ny) - ey(i);
        }
        fn(i, (unsigned)(R.off0 + gy * R.pitch + gx));
    }
}

// One coupled step of the 64 x TY tile `it` (the whole body of k_step; also the unit of
// work of the persistent batch kernel).  lane0 is zero: the persistent kernel passes an
// opaque zero so that the lane-index arithmetic stays inside its tile loop instead of
// being hoisted (and held in registers) across it.
template <class S, int TY, bool NT>
__device__ __forceinline__ void step_tile(const RunDev<S>* __restrict__ runs, const Item it,
                                          int parity, int first, int lane0) {
    __shared__ T s_rho[TY + 2][66];
    __shared__ T s_ux[TY + 2][66];
    __shared__ T s_uy[TY + 2][66];
    // wet-node walls: u_x, u_y and rho u_y^3 two rows into the fluid from the wall nodes
    // of the tile ([0] bottom wall, [1] top wall), for their one-sided differences
    __shared__ T s_w2[2][3][64];
    const RunDev<S>& R = runs[it.run];
    const S* src = R.pop[parity];
    S* dst = R.pop[parity ^ 1];
    const long long plane = R.plane;
    const bool pull = first == 0;
    const int lx = threadIdx.x + lane0, ly = threadIdx.y + lane0;
    const int tid = ly * 64 + lx;
    const int x0 = it.tx * 64, y0 = it.ty * TY;
    const int x = x0 + lx, y = y0 + ly;

    // ---- phase 1: own node (36 pulls, history, force) ----
    const bool in_dom = x < R.nx && y < R.ny;
    const int p = node_index(R, x, y);
    unsigned b = 0u;
    if (in_dom) b = node_bits(R, p);
    const bool active = in_dom && !(b & BIT_SELF_SOLID);
    if (active && wet_row(R, y)) {
        // recomputed from its pulled populations before this node's own pulls, so that
        // nothing extra stays live across them
        T r2 = 1.0, ux2 = 0.0, uy2 = 0.0;
        cell_macros(R, src, x, y == 0 ? 2 : y - 2, pull, r2, ux2, uy2);
        const int w = y == 0 ? 0 : 1;
        s_w2[w][0][lx] = ux2;
        s_w2[w][1][lx] = uy2;
        s_w2[w][2][lx] = r2 * uy2 * uy2 * uy2;
    }
    S f[9], g[3][9];
    T Fx = 0.0, Fy = 0.0;
    // history S(t-1), u(t-1), in storage precision until the collisions use it
    S hS[3] = {S(0), S(0), S(0)}, hux = S(0), huy = S(0);
    // conformation deviations A - I: the zeroth moments of the pulled g lattices (CNEBB
    // keeps them, so they are final before the wall reconstruction)
    T dk[3] = {0.0, 0.0, 0.0};
    if (active) {
        pull36(R, src, p, pull, f, g);
        if (pull && R.ylw && (b & 0x1FEu)) ylw_restore(R, src, p, b, f);
#pragma unroll
        for (int k = 0; k < 3; ++k) dk[k] = zeroth(g[k]);
        node_force(R, p, Fx, Fy);
        // wet-node wall: the populations from beyond the wall by non-equilibrium
        // bounce-back (the pulled ghost values are discarded)
        // (open end first, then the wall row: at a corner the wall rule has the last word)
        if (pull && nebb_end(R, x)) zou_he_x(f, x == 0, T(R.inlet[y]), Fx, Fy);
        if (pull && wet_row(R, y)) zou_he(f, y == 0, Fx, Fy);
        if (pull) hist_ld(R.hist, plane, (unsigned)p, hS, hux, huy);
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
        if (wet_row(R, y)) ux = uy = 0.0;  // wall node: the wall velocity
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
    // Neighbour values for the differences: LDS for fluid neighbours, the wall formula
    // at walls, inlet/outlet ghost values at open ends.  d(rho u^3) is taken before the
    // hydrodynamic collision (which uses it) and the velocity gradient after it (for the
    // conformation source), so that neither set of values is held across the other work.
    const bool wxl = (b >> 1) & 1u, wxh = (b >> 3) & 1u, wyl = (b >> 2) & 1u, wyh = (b >> 4) & 1u;
    const bool open_l = R.xmode == XM_OPEN && x == 0;
    const bool open_h = R.xmode == XM_OPEN && x == R.nx - 1;
    // wall fractions of the four axis links (1/2 on flat walls): low x, high x, low y, high y
    auto wall_q = [&](T q[4]) {
        q[0] = q[1] = q[2] = q[3] = 0.5;
        if (R.has_curved && (b & 0x1Eu)) {
            const int bi = R.bidx[p];
            q[0] = link_q(R, bi, 1); q[1] = link_q(R, bi, 3);
            q[2] = link_q(R, bi, 2); q[3] = link_q(R, bi, 4);
        }
    };
    // the four axis neighbours of rho (v = 0), u_x (1) or u_y (2)
    auto nbs = [&](int v, T& xl, T& xh, T& yl, T& yh) {
        auto fld = [&](int yy, int xx) -> T {
            return v == 0 ? s_rho[yy][xx] : (v == 1 ? s_ux[yy][xx] : s_uy[yy][xx]);
        };
        const T own = v == 0 ? rho : (v == 1 ? ux : uy);
        xl = open_l ? (v == 0 ? T(1.0) : (v == 1 ? T(R.inlet[y]) : T(0.0))) : (wxl ? 0.0 : fld(ly + 1, lx));
        xh = open_h ? own : (wxh ? 0.0 : fld(ly + 1, lx + 2));
        yl = wyl ? 0.0 : fld(ly, lx + 1);
        yh = wyh ? 0.0 : fld(ly + 2, lx + 1);
    };
    // wet-node wall row: wall-normal derivatives by the one-sided second-order
    // difference through the node and the next two rows (the nearer from the tile's LDS,
    // the farther from s_w2)
    const bool wet = wet_row(R, y);
    const int wsd = y == 0 ? 0 : 1;
    const T s1 = y == 0 ? 1.0 : -1.0;
    T Dx, Dy;
    {
        T q[4], rxl, rxh, ryl, ryh, axl, axh, ayl, ayh, bxl, bxh, byl, byh;
        wall_q(q);
        nbs(0, rxl, rxh, ryl, ryh);
        nbs(1, axl, axh, ayl, ayh);
        nbs(2, bxl, bxh, byl, byh);
        Dx = dgrad(wxl, q[0], rxl * axl * axl * axl, rho * ux * ux * ux, wxh, q[1], rxh * axh * axh * axh);
        Dy = dgrad(wyl, q[2], ryl * byl * byl * byl, rho * uy * uy * uy, wyh, q[3], ryh * byh * byh * byh);
        if (wet) {
            const T r1 = y == 0 ? ryh : ryl, uy1 = y == 0 ? byh : byl;
            Dy = s1 * (-1.5 * (rho * uy * uy * uy) + 2.0 * (r1 * uy1 * uy1 * uy1) -
                       0.5 * s_w2[wsd][2][lx]);
        }
    }
    const T d0 = dk[0], d1 = dk[1], d2 = dk[2];
    T txx, txy, tyy;
    {
        T rf[3] = {d0, d1, d2}, sf[3] = {d0, d1, d2};
        if (R.model != MODEL_OLDROYD_B) closure(R.model, R.mpar, d0, d1, d2, rf, sf);
        txx = R.eta_over_lam * sf[0], txy = R.eta_over_lam * sf[1], tyy = R.eta_over_lam * sf[2];
    }

    // Post-collision populations of the four lattices, in storage precision, stored
    // together at the end (one vector store per direction).  Until then f, g^xx and g^xy
    // wait in LDS, one column per lane (single-precision storage: registers are what
    // limits the step to four waves per SIMD), or in registers (double precision);
    // g^yy, computed last, stays in registers.
    constexpr bool kStage = sizeof(S) == 4;
    __shared__ S s_post[kStage ? 27 : 1][kStage ? 64 * TY : 1];
    S rpost[kStage ? 1 : 27];
    auto put = [&](int j, T v) {
        if constexpr (kStage) s_post[j][tid] = S(v);
        else rpost[j] = S(v);
    };
    auto get = [&](int j) -> S {
        if constexpr (kStage) return s_post[j][tid];
        else return rpost[j];
    };
    S g2[9];
    {
        T out[9];
        collide_hydro(R, moments(f), rho, ux, uy, Fx, Fy, txx, txy, tyy, Dx, Dy, out);
#pragma unroll
        for (int i = 0; i < 9; ++i) put(i, out[i]);
    }
    // velocity gradient, constitutive source S(t) and the history the next step needs
    T Sc[3];
    {
        T q[4], axl, axh, ayl, ayh, bxl, bxh, byl, byh;
        wall_q(q);
        nbs(1, axl, axh, ayl, ayh);
        nbs(2, bxl, bxh, byl, byh);
        const T Lxx = dgrad(wxl, q[0], axl, ux, wxh, q[1], axh);
        const T Lxy = dgrad(wxl, q[0], bxl, uy, wxh, q[1], bxh);
        T Lyx = dgrad(wyl, q[2], ayl, ux, wyh, q[3], ayh);
        T Lyy = dgrad(wyl, q[2], byl, uy, wyh, q[3], byh);
        if (wet) {
            const T ux1 = y == 0 ? ayh : ayl, uy1 = y == 0 ? byh : byl;
            Lyx = s1 * (-1.5 * ux + 2.0 * ux1 - 0.5 * s_w2[wsd][0][lx]);
            Lyy = s1 * (-1.5 * uy + 2.0 * uy1 - 0.5 * s_w2[wsd][1][lx]);
        }
        const T axx = 1.0 + d0, axy = d1, ayy = 1.0 + d2;
        T rf[3] = {d0, d1, d2}, sf[3] = {d0, d1, d2};
        if (R.model != MODEL_OLDROYD_B) closure(R.model, R.mpar, d0, d1, d2, rf, sf);
        if (R.no_source) {
            Sc[0] = Sc[1] = Sc[2] = 0.0;
        } else {
            const T d = Lxx + Lyy;
            Sc[0] = -R.inv_lam * rf[0] + 2.0 * (axx * Lxx + axy * Lyx) + axx * d;
            Sc[1] = -R.inv_lam * rf[1] + axx * Lxy + axy * Lyy + axy * Lxx + ayy * Lyx + axy * d;
            Sc[2] = -R.inv_lam * rf[2] + 2.0 * (axy * Lxy + ayy * Lyy) + ayy * d;
        }
    }
    hist_st<NT>(R.hist_out, plane, (unsigned)p, Sc, ux, uy);
    // conformation lattices one at a time after the hydrodynamic one (keeps the
    // register budget of four waves per SIMD): CNEBB at wall-adjacent nodes, moments,
    // collision
    const unsigned solid = pull ? (b & 0x1FEu) : 0u;
    const T inv_rho = 1.0 / rho;
    // F~(t - 1) of the collisions: from the history, or on the first step F~(t - 1) := F~(t)
    const T uxp = pull ? T(hux) : ux, uyp = pull ? T(huy) : uy;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Mom gm;
        if (solid) {
            T gg[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) gg[i] = T(g[k][i]);
            cnebb(solid, k, ux, uy, gg);
            gm = moments(gg);
        } else {
            gm = moments(g[k]);
        }
        gm.m0 = dk[k];
        const T phi = phi0(k) + dk[k];
        T out[9];
        collide_cde(R, gm, phi, ux, uy, phi * inv_rho, Fx, Fy, Sc[k], pull ? T(hS[k]) : Sc[k], uxp,
                    uyp, out);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (k < 2) put(9 + 9 * k + i, out[i]);
            else g2[i] = S(out[i]);
        }
    }
    auto post4 = [&](int i) -> V4<S> {
        V4<S> v;
        v.x = get(i);
        v.y = get(9 + i);
        v.z = get(18 + i);
        v.w = g2[i];
        return v;
    };
#pragma unroll
    for (int i = 0; i < 9; ++i) st4<NT>(dst, plane, i, (unsigned)p, post4(i));
    // Open ends (Sec. 4.3): the first (last) column node writes the ghosts its row's
    // inlet (outlet) links pull next step by non-equilibrium extrapolation from its own
    // post-collision populations (as stored): f_i = f_i^eq(rho_b, u_b) + f_i -
    // f_i^eq(rho, u) with rho, u their moments; inlet rho_b = rho, u_b = profile;
    // outlet rho_b = 1, u_b = u.  Conformation: inlet g_i = g_i^eq(A_in, u_in) + g_i -
    // g_i^eq(phi, u) with phi the moment of the stored g; outlet a copy (zero gradient).
    if (R.xmode == XM_OPEN && (x == 0 || x == R.nx - 1)) {
        const bool oin = x == 0;
        S fo[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) fo[i] = get(i);
        T odr, orho, oux, ouy;
        hydro_macros(fo, 0.0, 0.0, odr, orho, oux, ouy);
        const T uin = oin ? T(R.inlet[y]) : 0.0;
        T dphi[3], ain[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T acc = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) acc += T(k < 2 ? get(9 + 9 * k + i) : g2[i]);
            dphi[k] = acc;
            ain[k] = oin ? T(R.inlet[(1 + k) * R.ny + y]) : 0.0;
        }
        open_end_slots(R, y, oin, [&](int i, unsigned gs) {
            const V4<S> v = post4(i);
            const T fneq = T(v.x) - dfeq(i, odr, orho, oux, ouy);
            const T gk[3] = {T(v.y), T(v.z), T(v.w)};
            T gv[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                gv[k] = oin ? dgeq(i, ain[k] - phi0(k), ain[k], uin, 0.0) + gk[k] -
                                  dgeq(i, dphi[k], phi0(k) + dphi[k], oux, ouy)
                            : gk[k];
            st4<false>(dst, plane, i, gs,
                       make4<S>((oin ? dfeq(i, odr, orho, uin, 0.0) : dfeq(i, 0.0, 1.0, oux, ouy)) + fneq,
                                gv[0], gv[1], gv[2]));
        });
    }
    // Periodic images: an edge node also writes the populations that leave the domain
    // into the ghost slots its periodic neighbours pull from (no fill op needed).
    const bool px_per = R.xmode == XM_PERIODIC, py_per = R.ymode == XM_PERIODIC;
    const int gxo = (px_per && x == R.nx - 1) ? -R.nx : ((px_per && x == 0) ? R.nx : 0);
    const int gyo = (py_per && y == R.ny - 1) ? -R.ny : ((py_per && y == 0) ? R.ny : 0);
    if ((gxo | gyo) != 0) {
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            // a population moving in direction i leaves through the edge it points at
            const int sx = (gxo != 0 && ex(i) == (gxo < 0 ? 1 : -1)) ? gxo : 0;
            const int sy = (gyo != 0 && ey(i) == (gyo < 0 ? 1 : -1)) ? gyo : 0;
            if (sx == 0 && sy == 0) continue;
            st4<false>(dst, plane, i, (unsigned)(p + sx + sy * R.pitch), post4(i));
        }
    }
}

}  // namespace
}  // namespace vlb
