// Device helpers shared by the forward-step and adjoint kernels: lattice constants,
// equilibria, pulls, moments, the moment-form collisions and the finite differences.
// Header-only; every kernel source compiles its own copy with the same flags.
#pragma once
#include "vlb_internal.h"

#define VLB_GLOBAL __attribute__((address_space(1)))

namespace vlb {
namespace {


using T = double;  // arithmetic type

// load/store with a uniform base pointer and a non-negative 32-bit element offset
template <class S>
__device__ __forceinline__ T ldu(const S* base, unsigned off) {
    return (T)((const VLB_GLOBAL S*)base)[off];
}
template <class S>
__device__ __forceinline__ void stu(S* base, unsigned off, T v) {
    ((VLB_GLOBAL S*)base)[off] = (S)v;
}
// store of a streamed value, read by other workgroups in the next step only: a
// non-temporal store when the working set exceeds the last-level cache, a plain one
// when the whole state stays cache resident
template <bool NT, class S>
__device__ __forceinline__ void st_stream(S* base, unsigned off, T v) {
    if (NT) __builtin_nontemporal_store((S)v, (VLB_GLOBAL S*)base + off);
    else ((VLB_GLOBAL S*)base)[off] = (S)v;
}

// ---- state layout ----
// Population buffer: direction-major with the four lattices of a direction interleaved,
// (f_i, g^xx_i, g^xy_i, g^yy_i) as one 16-byte (FP32) or 32-byte (FP64) vector per slot:
// element (lattice L, direction i, slot) at (i * plane + slot) * 4 + L.  A pull of all
// four lattices in direction i is one vector load from one address stream, so a node
// reads 9 streams instead of 36.
// History buffer: (S_xx, S_xy, S_yy, u_x) of the previous step as one vector per slot
// (the first 4 planes' worth), then u_y as a scalar plane at 4 * plane.
template <class S> struct Vec4Of;
template <> struct Vec4Of<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec4Of<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <class S> using V4 = typename Vec4Of<S>::type;

template <class S>
__device__ __forceinline__ V4<S> ld4(const S* buf, long long plane, int i, unsigned slot) {
    return ((const VLB_GLOBAL V4<S>*)(buf + 4 * (long long)i * plane))[slot];
}
template <bool NT, class S>
__device__ __forceinline__ void st4(S* buf, long long plane, int i, unsigned slot, V4<S> v) {
    VLB_GLOBAL V4<S>* a = (VLB_GLOBAL V4<S>*)(buf + 4 * (long long)i * plane) + slot;
    if (NT) __builtin_nontemporal_store(v, a);
    else *a = v;
}
// one lattice's population (scalar access: ring cells, boundary ops, read-out)
template <class S>
__device__ __forceinline__ T ld1(const S* buf, long long plane, int L, int i, unsigned slot) {
    return (T)((const VLB_GLOBAL S*)(buf + 4 * (long long)i * plane))[4 * slot + (unsigned)L];
}
template <class S>
__device__ __forceinline__ V4<S> make4(T a, T b, T c, T d) {
    V4<S> v;
    v.x = (S)a;
    v.y = (S)b;
    v.z = (S)c;
    v.w = (S)d;
    return v;
}
// history of the previous step at a slot: S_xx, S_xy, S_yy, u_x, u_y (V = S keeps them
// in storage precision until used, V = T converts)
template <class S, class V>
__device__ __forceinline__ void hist_ld(const S* h, long long plane, unsigned slot, V hS[3], V& hux,
                                        V& huy) {
    const V4<S> v = ((const VLB_GLOBAL V4<S>*)h)[slot];
    hS[0] = (V)v.x;
    hS[1] = (V)v.y;
    hS[2] = (V)v.z;
    hux = (V)v.w;
    huy = (V)((const VLB_GLOBAL S*)(h + 4 * plane))[slot];
}
template <bool NT, class S>
__device__ __forceinline__ void hist_st(S* h, long long plane, unsigned slot, const T Sk[3], T ux,
                                        T uy) {
    const V4<S> v = make4<S>(Sk[0], Sk[1], Sk[2], ux);
    VLB_GLOBAL V4<S>* a = (VLB_GLOBAL V4<S>*)h + slot;
    if (NT) __builtin_nontemporal_store(v, a);
    else *a = v;
    st_stream<NT>(h + 4 * plane, slot, uy);
}

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
__device__ __forceinline__ constexpr T wgt(int i) {
    return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
constexpr T R3 = 1.0 / 3.0;

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp");

template <class S>
__device__ __forceinline__ int node_index(const RunDev<S>& R, int x, int y) {
    return R.off0 + y * R.pitch + x;
}

// Deviation of the third-order Hermite hydrodynamic equilibrium (Sec. 3.1):
// f_i^eq - w_i = w_i [drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u + 13.5 h3_i(u))].
__device__ __forceinline__ T dfeq(int i, T drho, T rho, T ux, T uy) {
    const T eu = T(ex(i)) * ux + T(ey(i)) * uy;
    const T hxxy = (T(ex(i) * ex(i)) - R3) * T(ey(i));
    const T hxyy = (T(ey(i) * ey(i)) - R3) * T(ex(i));
    const T h3 = hxxy * ux * ux * uy + hxyy * ux * uy * uy;
    return wgt(i) * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy) + 13.5 * h3));
}

// Deviation of the second-order convection-diffusion equilibrium (Sec. 3.2).
__device__ __forceinline__ T dgeq(int i, T dphi, T phi, T ux, T uy) {
    const T eu = T(ex(i)) * ux + T(ey(i)) * uy;
    return wgt(i) * (dphi + phi * (3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy)));
}

__device__ __forceinline__ constexpr T phi0(int k) { return k == 1 ? 0.0 : 1.0; }

template <class S>
__device__ __forceinline__ T link_q(const RunDev<S>& R, int bi, int i) {
    return bi >= 0 ? R.bq[bi * 8 + (i - 1)] : 0.5;
}

template <class S>
__device__ __forceinline__ unsigned node_bits(const RunDev<S>& R, int p) {
    return R.has_bits ? (unsigned)((const VLB_GLOBAL uint16_t*)R.bits)[p] : 0u;
}

template <class S>
__device__ __forceinline__ void node_force(const RunDev<S>& R, int p, T& Fx, T& Fy) {
    if (R.uniform_force) {
        Fx = R.Fx;
        Fy = R.Fy;
    } else {
        Fx = ldu(R.force, (unsigned)p);
        Fy = ldu(R.force + R.plane, (unsigned)p);
    }
}

// The nine populations of lattice L (0 hydro, 1..3 conformation) that arrive at slot
// p: pulled from p - e_i, or the node's own values on the first step.  Kept in storage
// precision until their moments are taken.
template <class S>
__device__ __forceinline__ void pull9(const RunDev<S>& R, const S* src, int L, int p, bool pull,
                                      S v[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int off = pull ? p - ex(i) - ey(i) * R.pitch : p;
        v[i] = (S)ld1(src, R.plane, L, i, (unsigned)off);
    }
}
// All 36 populations arriving at slot p: one vector load per direction.
template <class S>
__device__ __forceinline__ void pull36(const RunDev<S>& R, const S* src, int p, bool pull, S f[9],
                                       S g[3][9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int off = pull ? p - ex(i) - ey(i) * R.pitch : p;
        const V4<S> v = ld4(src, R.plane, i, (unsigned)off);
        f[i] = v.x;
        g[0][i] = v.y;
        g[1][i] = v.z;
        g[2][i] = v.w;
    }
}

// rho, u with the half-force shift (Sec. 3.1).
template <class V>
__device__ __forceinline__ void hydro_macros(const V f[9], T Fx, T Fy, T& drho, T& rho, T& ux,
                                             T& uy) {
    const T s13 = T(f[1]) + T(f[3]), s24 = T(f[2]) + T(f[4]);
    const T s57 = T(f[5]) + T(f[7]), s68 = T(f[6]) + T(f[8]);
    const T d13 = T(f[1]) - T(f[3]), d24 = T(f[2]) - T(f[4]);
    const T d57 = T(f[5]) - T(f[7]), d68 = T(f[6]) - T(f[8]);
    drho = T(f[0]) + (s13 + s24) + (s57 + s68);
    const T jx = d13 + (d57 - d68), jy = d24 + (d57 + d68);
    rho = 1.0 + drho;
    const T inv = 1.0 / rho;
    ux = (jx + 0.5 * Fx) * inv;
    uy = (jy + 0.5 * Fy) * inv;
}

// Wall node of a wet-node wall (first or last row).
template <class S>
__device__ __forceinline__ bool wet_row(const RunDev<S>& R, int y) {
    return R.wet_y && (y == 0 || y == R.ny - 1);
}

// Non-equilibrium bounce-back of the hydrodynamic populations at a wet-node wall node
// (Zou-He closure with zero wall velocity): the three populations that would arrive
// from beyond the wall are set so that the node keeps the normal non-equilibrium part
// of its opposite and the streamed momentum equals -F/2 (zero velocity with the
// half-force shift).  The relations are differences of equally weighted populations,
// so they hold for the deviations f_i - w_i as stored.
// (Both candidate sets are formed and selected per entry, so that every array index
// stays a compile-time constant and f stays in registers.)
template <class V>
__device__ __forceinline__ void zou_he(V f[9], bool bottom, T Fx, T Fy) {
    const T jx = -0.5 * Fx, jy = -0.5 * Fy;
    const T d13 = T(f[1]) - T(f[3]);
    // bottom wall, unknown e_y = +1
    const V b2 = V(T(f[4]) + (2.0 / 3.0) * jy);
    const V b5 = V(T(f[7]) - 0.5 * d13 + (1.0 / 6.0) * jy + 0.5 * jx);
    const V b6 = V(T(f[8]) + 0.5 * d13 + (1.0 / 6.0) * jy - 0.5 * jx);
    // top wall, unknown e_y = -1
    const V t4 = V(T(f[2]) - (2.0 / 3.0) * jy);
    const V t7 = V(T(f[5]) + 0.5 * d13 - (1.0 / 6.0) * jy - 0.5 * jx);
    const V t8 = V(T(f[6]) - 0.5 * d13 - (1.0 / 6.0) * jy + 0.5 * jx);
    f[2] = bottom ? b2 : f[2];
    f[5] = bottom ? b5 : f[5];
    f[6] = bottom ? b6 : f[6];
    f[4] = bottom ? f[4] : t4;
    f[7] = bottom ? f[7] : t7;
    f[8] = bottom ? f[8] : t8;
}

// Wet-node NEBB open end (Sec. 4.3, the hydrodynamic inlet and outlet of the cylinder):
// at the first column the three populations from beyond the inlet (e_x = +1) for the
// prescribed velocity (uin, 0), at the last column those from beyond the outlet
// (e_x = -1) for density 1 and u_y = 0, by the Zou-He closure: the normal unknown keeps
// the non-equilibrium part of its opposite, the diagonals close the x and y momentum.
// The streamed momentum is j = rho u - F/2 (half-force shift).  The inlet density comes
// from the known populations, rho = (K - F_x/2) / (1 - uin) with K the rest, tangential
// and twice the outgoing populations; the outlet momentum is j_x = K - 1.  On the stored
// deviations f_i - w_i the weights of K sum to 1, and every other relation is a
// difference of equally weighted populations.
template <class V>
__device__ __forceinline__ void zou_he_x(V f[9], bool inlet, T uin, T Fx, T Fy) {
    const T jy = -0.5 * Fy;
    const T d24 = T(f[2]) - T(f[4]);
    const T c = T(f[0]) + T(f[2]) + T(f[4]);
    // inlet, unknown e_x = +1
    const T Ki = c + 2.0 * (T(f[3]) + T(f[6]) + T(f[7]));
    const T rho = (1.0 + Ki - 0.5 * Fx) / (1.0 - uin);
    const T jxi = rho * uin - 0.5 * Fx;
    const V i1 = V(T(f[3]) + (2.0 / 3.0) * jxi);
    const V i5 = V(T(f[7]) - 0.5 * d24 + (1.0 / 6.0) * jxi + 0.5 * jy);
    const V i8 = V(T(f[6]) + 0.5 * d24 + (1.0 / 6.0) * jxi - 0.5 * jy);
    // outlet, unknown e_x = -1
    const T jxo = c + 2.0 * (T(f[1]) + T(f[5]) + T(f[8]));
    const V o3 = V(T(f[1]) - (2.0 / 3.0) * jxo);
    const V o7 = V(T(f[5]) + 0.5 * d24 - (1.0 / 6.0) * jxo - 0.5 * jy);
    const V o6 = V(T(f[8]) - 0.5 * d24 - (1.0 / 6.0) * jxo + 0.5 * jy);
    f[1] = inlet ? i1 : f[1];
    f[5] = inlet ? i5 : f[5];
    f[8] = inlet ? i8 : f[8];
    f[3] = inlet ? f[3] : o3;
    f[7] = inlet ? f[7] : o7;
    f[6] = inlet ? f[6] : o6;
}

// The node is a wet NEBB open-end node.
template <class S>
__device__ __forceinline__ bool nebb_end(const RunDev<S>& R, int x) {
    return R.open_nebb && (x == 0 || x == R.nx - 1);
}

// Conservative non-equilibrium bounce-back for one lattice at a boundary node
// (Sec. 3.3).  On entry g holds the known post-streaming populations and, on wall
// links, the post-collision populations that moved toward the wall; phi_b is their
// sum.  Unknowns are rebuilt from the equilibrium at (phi_b, u_b) plus the
// non-equilibrium part of the known opposite population (the equilibrium alone when
// the opposite is unknown too); g_0 restores phi_b exactly.
// An unknown is never read as the known opposite of another unknown, so the update is
// done in place.
__device__ __forceinline__ void cnebb(unsigned solid, int k, T ux, T uy, T g[9]) {
    T sum = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) sum += g[i];
    const T phi = phi0(k) + sum;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (!((solid >> i) & 1u)) continue;
        const int o = opp(i);
        T v = dgeq(i, sum, phi, ux, uy);
        if (!((solid >> o) & 1u)) v += g[o] - dgeq(o, sum, phi, ux, uy);
        g[i] = v;
    }
    T rest = sum;
#pragma unroll
    for (int i = 1; i < 9; ++i) rest -= g[i];
    g[0] = rest;
}

// Finite-difference derivative along one axis: central difference, or the quadratic
// through the no-slip wall value 0 at fraction q when a neighbour is a wall.
__device__ __forceinline__ T dgrad(bool lo_wall, T qlo, T vlo, T v0, bool hi_wall, T qhi, T vhi) {
    if (!lo_wall && !hi_wall) return 0.5 * (vhi - vlo);
    if (lo_wall && !hi_wall) return qlo / (1.0 + qlo) * vhi + (1.0 - qlo) / qlo * v0;
    if (!lo_wall) return -(qhi / (1.0 + qhi) * vlo + (1.0 - qhi) / qhi * v0);
    return v0 * (qhi - qlo) / (qlo * qhi);
}

// Constitutive closure at one node from B = A - I (b0 = B_xx, b1 = B_xy, b2 = B_yy):
// the relaxation function F_r of the conformation equation and the stress function
// F_s of the Kramers relation (Sec. 2.2); Oldroyd-B is F_r = F_s = B.  The model is
// uniform per run, so the branch is too.  mp: alpha (Giesekus), eps (PTT), L^2 - 2
// (FENE-P, written as f A - I = (f - 1)(I + B) + B with f - 1 = tr B / (L^2 - 2 - tr B)).
__device__ __forceinline__ void closure(int model, T mp, T b0, T b1, T b2, T r[3], T s[3]) {
    r[0] = s[0] = b0;
    r[1] = s[1] = b1;
    r[2] = s[2] = b2;
    if (model == MODEL_GIESEKUS) {
        r[0] = b0 + mp * (b0 * b0 + b1 * b1);
        r[1] = b1 + mp * b1 * (b0 + b2);
        r[2] = b2 + mp * (b1 * b1 + b2 * b2);
    } else if (model == MODEL_LPTT || model == MODEL_EPTT) {
        const T x = mp * (b0 + b2);
        const T Y = model == MODEL_LPTT ? 1.0 + x : exp(x);
        r[0] = Y * b0;
        r[1] = Y * b1;
        r[2] = Y * b2;
    } else if (model == MODEL_FENE_P) {
        const T tr = b0 + b2;
        const T fm1 = tr / (mp - tr);
        r[0] = s[0] = fm1 * (1.0 + b0) + b0;
        r[1] = s[1] = (1.0 + fm1) * b1;
        r[2] = s[2] = fm1 * (1.0 + b2) + b2;
    }
}

// Moments of one D2Q9 population set via opposite-pair sums and differences:
// zeroth, first (x, y), second (xx, yy, xy) and the two third-order ones (xxy, xyy).
struct Mom {
    T m0, mx, my, pxx, pyy, pxy, qxxy, qxyy;
};
// Transpose of the closure's Jacobian (the adjoint of closure() above): for weights wr
// on F_r and ws on F_s, out_j = sum_i wr_i dF_r,i/db_j + ws_i dF_s,i/db_j with
// b = (B_xx, B_xy, B_yy) as closure() takes it.
__device__ __forceinline__ void closure_adj(int model, T mp, T b0, T b1, T b2, const T wr[3],
                                            const T ws[3], T out[3]) {
    out[0] = wr[0] + ws[0];
    out[1] = wr[1] + ws[1];
    out[2] = wr[2] + ws[2];
    if (model == MODEL_GIESEKUS) {
        out[0] = wr[0] * (1.0 + 2.0 * mp * b0) + wr[1] * (mp * b1) + ws[0];
        out[1] = (wr[0] + wr[2]) * (2.0 * mp * b1) + wr[1] * (1.0 + mp * (b0 + b2)) + ws[1];
        out[2] = wr[1] * (mp * b1) + wr[2] * (1.0 + 2.0 * mp * b2) + ws[2];
    } else if (model == MODEL_LPTT || model == MODEL_EPTT) {
        const T x = mp * (b0 + b2);
        const T Y = model == MODEL_LPTT ? 1.0 + x : exp(x);
        const T dY = model == MODEL_LPTT ? mp : mp * Y;  // dY/db_xx = dY/db_yy
        const T wb = wr[0] * b0 + wr[1] * b1 + wr[2] * b2;
        out[0] = Y * wr[0] + dY * wb + ws[0];
        out[1] = Y * wr[1] + ws[1];
        out[2] = Y * wr[2] + dY * wb + ws[2];
    } else if (model == MODEL_FENE_P) {
        const T tr = b0 + b2;
        const T den = mp - tr;
        const T fm1 = tr / den;
        const T dfm = mp / (den * den);  // d(f - 1)/db_xx = d(f - 1)/db_yy
        const T w0 = wr[0] + ws[0], w1 = wr[1] + ws[1], w2 = wr[2] + ws[2];
        const T wI = w0 * (1.0 + b0) + w1 * b1 + w2 * (1.0 + b2);
        out[0] = (1.0 + fm1) * w0 + dfm * wI;
        out[1] = (1.0 + fm1) * w1;
        out[2] = (1.0 + fm1) * w2 + dfm * wI;
    }
}

// One boundary-fill op on the post-collision buffer buf (see FillOp): write into the
// ghost or solid slot op.dst the value that the fluid node op.src pulls in direction
// dir next step.
template <class S>
__device__ __forceinline__ void apply_fill_op(const RunDev<S>& R, const FillOp& op, S* buf) {
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
        T a[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T ak = in ? T(R.inlet[(1 + k) * R.ny + op.far]) : phi0(k);
            a[k] = in ? dgeq(dir, ak - phi0(k), ak, uin, 0.0) : 0.0;
        }
        st4<false>(buf, plane, dir, (unsigned)op.dst,
                   make4<S>(in ? dfeq(dir, 0.0, 1.0, uin, 0.0) : 0.0, a[0], a[1], a[2]));
    } else {
        // conformation lattices: the populations that left toward the wall (CNEBB input);
        // hydrodynamic lattice: half-way or linear interpolated bounce-back
        V4<S> v = ld4(buf, plane, o, (unsigned)op.src);
        if (kind == FILL_CURVED && R.ylw) {
            // YLW (Sec. 4.3): the population that left toward the wall, interpolated to the
            // wall point between where direction o sits after streaming (the node, from
            // the far node x + e_dir; the solid, from the node), bounced, and
            // interpolated back to the node with the direction-dir population streamed
            // one spacing away from the wall: [(1 - q) f_o(far) + q f_o(x) + q f_dir(x)]
            // / (1 + q).  Half-way without a fluid far node.
            if (op.far >= 0) {
                const T q = op.q;
                v.x = S(((1.0 - q) * T(ld1(buf, plane, 0, o, (unsigned)op.far)) + q * T(v.x) +
                         q * T(ld1(buf, plane, 0, dir, (unsigned)op.src))) / (1.0 + q));
            }
        } else if (kind == FILL_CURVED) {
            const T q = op.q, fo = T(v.x);
            if (q < 0.5) {
                if (op.far >= 0) v.x = S(2.0 * q * fo + (1.0 - 2.0 * q) * ld1(buf, plane, 0, o, (unsigned)op.far));
            } else {
                v.x = S(fo / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * ld1(buf, plane, 0, dir, (unsigned)op.src));
            }
        }
        st4<false>(buf, plane, dir, (unsigned)op.dst, v);
    }
}

// Zeroth moment with the same pairing and rounding as Mom::m0 below.
template <class V>
__device__ __forceinline__ T zeroth(const V v[9]) {
    return T(v[0]) + ((T(v[1]) + T(v[3])) + (T(v[2]) + T(v[4]))) +
           ((T(v[5]) + T(v[7])) + (T(v[6]) + T(v[8])));
}
template <class V>
__device__ __forceinline__ Mom moments(const V v[9]) {
    const T s13 = T(v[1]) + T(v[3]), d13 = T(v[1]) - T(v[3]);
    const T s24 = T(v[2]) + T(v[4]), d24 = T(v[2]) - T(v[4]);
    const T s57 = T(v[5]) + T(v[7]), d57 = T(v[5]) - T(v[7]);
    const T s68 = T(v[6]) + T(v[8]), d68 = T(v[6]) - T(v[8]);
    Mom m;
    m.m0 = T(v[0]) + (s13 + s24) + (s57 + s68);
    m.mx = d13 + (d57 - d68);
    m.my = d24 + (d57 + d68);
    m.pxx = s13 + (s57 + s68);
    m.pyy = s24 + (s57 + s68);
    m.pxy = s57 - s68;
    m.qxxy = d57 + d68;
    m.qxyy = d57 - d68;
    return m;
}

// Populations w_i [e0 + 3 e.M1 + 4.5 H2:M2 + 13.5 H3:M3] rebuilt pairwise: for the
// opposite directions i and i' the even part is shared and the odd part changes sign.
__device__ __forceinline__ void rebuild(T e0, T m1x, T m1y, T m2xx, T m2yy, T m2xy, T m3xxy,
                                        T m3xyy, T out[9]) {
    constexpr T w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w5 = 1.0 / 36.0;
    const T tr = m2xx + m2yy;
    out[0] = w0 * (e0 - 1.5 * tr);
    const T e13 = e0 + 3.0 * m2xx - 1.5 * m2yy, o13 = 3.0 * m1x - 4.5 * m3xyy;
    out[1] = w1 * (e13 + o13);
    out[3] = w1 * (e13 - o13);
    const T e24 = e0 + 3.0 * m2yy - 1.5 * m2xx, o24 = 3.0 * m1y - 4.5 * m3xxy;
    out[2] = w1 * (e24 + o24);
    out[4] = w1 * (e24 - o24);
    const T ed = e0 + 3.0 * tr;
    const T e57 = ed + 9.0 * m2xy, o57 = 3.0 * (m1x + m1y) + 9.0 * (m3xxy + m3xyy);
    out[5] = w5 * (e57 + o57);
    out[7] = w5 * (e57 - o57);
    const T e68 = ed - 9.0 * m2xy, o68 = 3.0 * (m1y - m1x) + 9.0 * (m3xxy - m3xyy);
    out[6] = w5 * (e68 + o68);
    out[8] = w5 * (e68 - o68);
}

// Hydrodynamic TRT regularized collision in Hermite-moment form (Sec. 3.1): the
// post-collision populations are w_i [drho + 3 e.M1 + 4.5 H2:M2 + 13.5 H3:M3] with
//   M1 = rho u + (1 - 1/tau_s1) a_1 + (1 - 1/(2 tau_s1)) F                      (F_i)
//   M2 = rho uu + (1 - 1/tau_s1) a_2 - (1 - 1/(2 tau_s1)) diag(Dx, Dy) - tau/tau_s1
//        (G_i and T_i)
//   M3 = rho uuu + (1 - 1/tau_s2) a_3   (xxy and xyy; H_xxx = H_yyy = 0 on D2Q9)
// where a_n are the off-equilibrium Hermite moments of f (a_0 = 0 identically).
template <class S>
__device__ __forceinline__ void collide_hydro(const RunDev<S>& R, const Mom& m, T rho, T ux, T uy,
                                              T Fx, T Fy, T txx, T txy, T tyy, T Dx, T Dy,
                                              T out[9]) {
    const T drho = m.m0;
    const T ruxx = rho * ux * ux, ruyy = rho * uy * uy, ruxy = rho * ux * uy;
    const T ax = m.mx - rho * ux, ay = m.my - rho * uy;
    const T axx = m.pxx - R3 * drho - ruxx;
    const T ayy = m.pyy - R3 * drho - ruyy;
    const T axy = m.pxy - ruxy;
    const T axxy = m.qxxy - R3 * m.my - ruxx * uy;
    const T axyy = m.qxyy - R3 * m.mx - ruyy * ux;
    const T m1x = rho * ux + R.c1 * ax + R.h1 * Fx;
    const T m1y = rho * uy + R.c1 * ay + R.h1 * Fy;
    const T m2xx = ruxx + R.c1 * axx - R.h1 * Dx - R.inv_ts1 * txx;
    const T m2yy = ruyy + R.c1 * ayy - R.h1 * Dy - R.inv_ts1 * tyy;
    const T m2xy = ruxy + R.c1 * axy - R.inv_ts1 * txy;
    const T m3xxy = ruxx * uy + R.c2 * axxy;
    const T m3xyy = ruyy * ux + R.c2 * axyy;
    rebuild(drho, m1x, m1y, m2xx, m2yy, m2xy, m3xxy, m3xyy, out);
}

// Convection-diffusion TRT regularized collision in moment form (Sec. 3.2):
// w_i [dphi + 1.5 S - 0.5 S_prev + 3 e.N1 + 4.5 H2:N2] with
//   N1 = phi u + (1 - 1/tau_p1) b_1 + (1 - 1/(2 tau_p1)) (F phi/rho + 1.5 S u - 0.5 S_prev u_prev)
//   N2 = phi uu + (1 - 1/tau_p2) b_2,
// i.e. the equilibrium, the regularized non-equilibrium part, G~_i, F~_i and half the
// backward time difference of F~_i.
template <class S>
__device__ __forceinline__ void collide_cde(const RunDev<S>& R, const Mom& m, T phi, T ux, T uy,
                                            T fr, T Fx, T Fy, T Sk, T Sp, T uxp, T uyp,
                                            T out[9]) {
    const T dphi = m.m0;
    const T pux = phi * ux, puy = phi * uy;
    const T bx = m.mx - pux, by = m.my - puy;
    const T bxx = m.pxx - R3 * dphi - pux * ux;
    const T byy = m.pyy - R3 * dphi - puy * uy;
    const T bxy = m.pxy - pux * uy;
    const T s0 = dphi + 1.5 * Sk - 0.5 * Sp;
    const T n1x = pux + R.p1 * bx + R.h2 * (Fx * fr + 1.5 * Sk * ux - 0.5 * Sp * uxp);
    const T n1y = puy + R.p1 * by + R.h2 * (Fy * fr + 1.5 * Sk * uy - 0.5 * Sp * uyp);
    const T n2xx = pux * ux + R.p2 * bxx;
    const T n2yy = puy * uy + R.p2 * byy;
    const T n2xy = pux * uy + R.p2 * bxy;
    rebuild(s0, n1x, n1y, n2xx, n2yy, n2xy, 0.0, 0.0, out);
}

// Periodic image of a tile/ring cell; false when it lies beyond a wall or open end.
template <class S>
__device__ __forceinline__ bool wrap_cell(const RunDev<S>& R, int& xx, int& yy) {
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

// Mass restore of the curved-wall scheme YLW (Sec. 4.3, with the conservation strategy
// CNEBB shares with it, Sec. 3.3): the rest population of a node with wall links takes
// what the wall fill did not return, so that the node holds its known populations plus
// those that left toward the wall -- its own post-collision values, still in its slot of
// src.  Stored values are deviations from w_i rho0 and opposite directions share a
// weight, so the difference is the same in either form.  Half-way links add exactly 0.
template <class S>
__device__ __forceinline__ void ylw_restore(const RunDev<S>& R, const S* src, int p, unsigned b,
                                            S f[9]) {
    T acc = T(f[0]);
#pragma unroll
    for (int d = 1; d < 9; ++d)
        if ((b >> d) & 1u) acc += T(ld1(src, R.plane, 0, opp(d), (unsigned)p)) - T(f[d]);
    f[0] = S(acc);
}

// rho and u of one tile/ring cell (hydrodynamic pull + moments); false if not fluid.
template <class S>
__device__ __forceinline__ bool cell_macros(const RunDev<S>& R, const S* src, int cx, int cy,
                                            bool pull, T& rho, T& ux, T& uy) {
    if (!wrap_cell(R, cx, cy)) return false;
    const int p = node_index(R, cx, cy);
    const unsigned b = node_bits(R, p);
    if (b & BIT_SELF_SOLID) return false;
    S f[9];
    pull9(R, src, 0, p, pull, f);
    if (pull && R.ylw && (b & 0x1FEu)) ylw_restore(R, src, p, b, f);
    T Fx, Fy, drho;
    node_force(R, p, Fx, Fy);
    const bool wet = wet_row(R, cy);
    if (pull && nebb_end(R, cx)) zou_he_x(f, cx == 0, T(R.inlet[cy]), Fx, Fy);
    if (wet && pull) zou_he(f, cy == 0, Fx, Fy);
    hydro_macros(f, Fx, Fy, drho, rho, ux, uy);
    if (wet) ux = uy = 0.0;  // wall node: the wall velocity
    return true;
}


}  // namespace
}  // namespace vlb
