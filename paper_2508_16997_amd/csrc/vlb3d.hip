// vlb3d.hip -- the coupled step in three dimensions (D3Q19 or D3Q27) for gfx950, and its
// C ABI (include/vlb3d.h).
//
// State: two population buffers of 7 q planes (7 lattices x q directions; plane
// (L * q + i), node (z * ny + y) * nx + x), storing deviations from the rest state
// (f_i - w_i, g_i - w_i phi0 with phi0 = 1 for A_xx, A_yy, A_zz and 0 otherwise); history
// of S (6 planes) and u (3 planes); rho and u at time n (4 planes) for the neighbours'
// differences; with solid nodes a plane of per-node link bits.  Per step two launches:
//   k3_macro  rho and u of every node from its pulled populations (mac planes)
//   k3_step   per node: pulls of all seven lattices (the conformation populations held in
//             registers in FP32 storage -- four of the six lattices on D3Q27 -- and
//             pulled again for the collision otherwise), the
//             conformation's zeroth moments, the velocity gradient from the mac planes of
//             the six axis neighbours, the constitutive source, the hydrodynamic collision
//             (stored at once), then lattice by lattice CNEBB at wall-adjacent nodes and
//             the conformation collision (stored at once); history in place.
// Pull streaming: node x takes direction i from x - e_i (periodic wrap in x and z, and in
// y unless walls); a source beyond a wall or a solid source gives the node's own
// post-collision value of the opposite direction (half-way bounce-back for f, the CNEBB
// input for g).
// One node per lane, one 64-lane row (one wave) per block, one z slice per block row.
// All arithmetic in double.
//
// The file is compiled twice: as itself (VLB3_PART 1: the FP32 kernels and the C ABI)
// and through vlb3d_f64.hip (VLB3_PART 2: the FP64 kernels behind three functions of
// namespace vlb3_f64), so that the two halves of the kernel set build side by side.
#ifndef VLB3_PART
#define VLB3_PART 1
#endif
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "vlb3d.h"
#include "vlb_internal.h"

namespace vlb3 {
namespace {

using T = double;
constexpr int NLAT = 7;  // hydrodynamic + six conformation lattices
// Block: TX x TY lanes, one wave per row.  One row per block measured fastest on the
// 2^22-node channel (D3Q19 1049, 1065, 1068 and 1164 us per step for TY = 1, 2, 4, 8;
// D3Q27 1517, 1539, 1558, 1705 us).
#ifndef VLB3_TY
#define VLB3_TY 1
#endif
constexpr int TX = 64, TY = VLB3_TY;
// Conformation lattices whose pulled populations k3_step holds in registers from the
// zeroth-moment pass to the collision (the others are pulled twice).  FP32 storage: all
// six on D3Q19 (two waves per SIMD, no second read), four of six on D3Q27 (the most
// that keeps two waves; measured 1723, 1643, 1607 and 1566 us per step on the 2^22-node
// channel for none, two, three and four).  FP64: none, where holding them would leave
// one wave per SIMD.
// With solid nodes (general unknown sets in CNEBB) one lattice fewer on D3Q19 and two
// fewer on D3Q27 keep two waves; a closure other than Oldroyd-B (its extra arithmetic)
// holds one lattice fewer again.
template <class S, class Lat, bool SOLIDS = false, bool CLOSURE = false>
constexpr int kHold = sizeof(S) == 4 ? (SOLIDS ? (Lat::Q == 19 ? 5 - CLOSURE : 2 - CLOSURE)
                                               : (Lat::Q == 19 ? 6 - CLOSURE : 4 - CLOSURE))
                                     : 0;
constexpr T CS2 = 1.0 / 3.0;

// conformation components: (a, b) of component k, rest value phi0
__host__ __device__ constexpr int ka(int k) { return k < 3 ? 0 : (k < 5 ? 1 : 2); }
__host__ __device__ constexpr int kb(int k) { return k == 0 ? 0 : (k == 1 || k == 3) ? 1 : 2; }
__host__ __device__ constexpr T phi0(int k) { return (k == 0 || k == 3 || k == 5) ? 1.0 : 0.0; }
// Velocities come in opposite pairs (2j - 1, 2j) after the rest velocity 0.
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// D3Q19 velocities: rest; +-x, +-y, +-z; the twelve face diagonals.
__host__ __device__ constexpr int e19(int i, int a) {
    return a == 0 ? ((i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
                     : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0)
         : a == 1 ? ((i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
                     : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0)
                  : ((i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
                     : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0);
}
// H_aab with a != b: e_a^2 e_b - c_s^2 e_b (H_abc = e_a e_b e_c - c_s^2 (e_a d_bc + e_b d_ac
// + e_c d_ab)).
__host__ __device__ constexpr T h3aab(int ea, int eb) { return (T)(ea * ea * eb) - CS2 * (T)eb; }

// D3Q19.  Third order (no H_aaa, no H_xyz on this lattice): the six combinations
// h_{c,s} = H_aab + s H_bcc for (a, b, c) = (x, y, z), (z, x, y), (y, z, x), basis index
// m = 2c (s = +1) and 2c + 1 (s = -1), orthogonal with lattice norms 2 c_s^6 and 6 c_s^6;
// the equilibrium's coefficient of h_{c,s} per unit density is u_a^2 u_b + s u_b u_c^2.
struct D3Q19 {
    static constexpr int Q = 19, NB3 = 6;
    __host__ __device__ static constexpr int e(int i, int a) { return e19(i, a); }
    __host__ __device__ static constexpr T w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int ca(int c) { return c == 0 ? 0 : (c == 1 ? 2 : 1); }
    __host__ __device__ static constexpr int cb(int c) { return c == 0 ? 1 : (c == 1 ? 0 : 2); }
    __host__ __device__ static constexpr int cc(int c) { return c == 0 ? 2 : (c == 1 ? 1 : 0); }
    __host__ __device__ static constexpr T h3(int i, int m) {
        return h3aab(e(i, ca(m >> 1)), e(i, cb(m >> 1))) +
               ((m & 1) ? -1.0 : 1.0) * h3aab(e(i, cc(m >> 1)), e(i, cb(m >> 1)));
    }
    __host__ __device__ static constexpr T h3inv(int m) { return (m & 1) ? 4.5 : 13.5; }
    __host__ __device__ static T u3(int m, const T u[3]) {
        const int a = ca(m >> 1), b = cb(m >> 1), c = cc(m >> 1);
        const T t1 = u[a] * u[a] * u[b], t2 = u[b] * u[c] * u[c];
        return (m & 1) ? t1 - t2 : t1 + t2;
    }
};

// D3Q27: the D3Q19 velocities, then the eight corners in opposite pairs -- (+,+,+),
// (+,+,-), (+,-,+), (-,+,+) at odd indices 19-25, their negatives after them.  Weights are
// products of the D1Q3 weights 2/3 and 1/6.  Third order: the six H_aab (a != b; basis
// index m for (a, b) = (x, y), (x, z), (y, x), (y, z), (z, x), (z, y)) and H_xyz (m = 6),
// orthogonal with their continuous norms 2 c_s^6 and c_s^6; equilibrium coefficients
// per unit density u_a^2 u_b and u_x u_y u_z.
struct D3Q27 {
    static constexpr int Q = 27, NB3 = 7;
    __host__ __device__ static constexpr int e(int i, int a) {
        return i < 19 ? e19(i, a)
                      : ((i & 1) ? 1 : -1) * ((((i - 19) >> 1) != 0 && a == 3 - ((i - 19) >> 1)) ? -1 : 1);
    }
    __host__ __device__ static constexpr T w(int i) {
        return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
    }
    __host__ __device__ static constexpr int ma(int m) { return m >> 1; }
    __host__ __device__ static constexpr int mb(int m) { return (m >> 1) == 0 ? 1 + (m & 1) : ((m >> 1) == 1 ? 2 * (m & 1) : (m & 1)); }
    __host__ __device__ static constexpr T h3(int i, int m) {
        return m == 6 ? (T)(e(i, 0) * e(i, 1) * e(i, 2)) : h3aab(e(i, ma(m)), e(i, mb(m)));
    }
    __host__ __device__ static constexpr T h3inv(int m) { return m == 6 ? 27.0 : 13.5; }
    __host__ __device__ static T u3(int m, const T u[3]) {
        return m == 6 ? u[0] * u[1] * u[2] : u[ma(m)] * u[ma(m)] * u[mb(m)];
    }
};

template <class S>
struct Run3 {
    int nx, ny, nz, ywall, first;
    int N;  // plane stride in elements (the node count rounded up, plus a pad)
    const S* src;
    S* dst;
    S* hist;  // 9 planes: S_xx, S_xy, S_xz, S_yy, S_yz, S_zz, u_x, u_y, u_z (previous step)
    S* mac;   // 4 planes: rho, u_x, u_y, u_z at time n
    const unsigned* bits;  // per node (solid nodes present): bit i = the pull of direction i
                           // comes from a solid node, bit 31 = the node is solid
    T c1, c2, h1, inv_ts1;  // hydrodynamic: 1 - 1/tau_s1, 1 - 1/tau_s2, 1 - 1/(2 tau_s1), 1/tau_s1
    T p1, p2, h2;           // conformation: 1 - 1/tau_p1, 1 - 1/tau_p2, 1 - 1/(2 tau_p1)
    T inv_lam, eta_over_lam, F[3];
    int no_source;
    int model;  // constitutive closure (VLB_OLDROYD_B ... VLB_FENE_P) and its parameter
    T mpar;
};

// c0 + e_i.c + e_i.M.e_i for the symmetric M stored as (xx, xy, xz, yy, yz, zz): with
// components of e_i in {-1, 0, 1} this is a handful of additions per direction.
template <class Lat>
__device__ __forceinline__ T quad_at(int i, T c0, const T c[3], const T M[6]) {
    T v = c0;
    const int e0 = Lat::e(i, 0), e1 = Lat::e(i, 1), e2 = Lat::e(i, 2);
    if (e0) v += e0 > 0 ? c[0] : -c[0];
    if (e1) v += e1 > 0 ? c[1] : -c[1];
    if (e2) v += e2 > 0 ? c[2] : -c[2];
    if (e0) v += M[0];
    if (e1) v += M[3];
    if (e2) v += M[5];
    if (e0 * e1) v += e0 * e1 > 0 ? 2.0 * M[1] : -2.0 * M[1];
    if (e0 * e2) v += e0 * e2 > 0 ? 2.0 * M[2] : -2.0 * M[2];
    if (e1 * e2) v += e1 * e2 > 0 ? 2.0 * M[4] : -2.0 * M[4];
    return v;
}

// Where node (x, y, z) pulls from: its own slot n and, per axis, the slot offsets of
// the source behind it for e = +1 ([0]) and e = -1 ([1]) with the periodic wrap; the wall
// flags mark rows whose pulls from beyond y are the node's own opposite values.  On the
// first step every pull is the node's own slot (the initial state sits there).
struct Nbr {
    int n;
    int dx[2], dy[2], dz[2];
    bool ylo_wall, yhi_wall, first;
    unsigned sol;  // directions whose pull comes from a solid node (0 without solids)
};
constexpr unsigned SELF_SOLID = 1u << 31;
template <class S>
__device__ __forceinline__ Nbr make_nbr(const Run3<S>& R, int x, int y, int z) {
    Nbr b;
    const int nxy = R.nx * R.ny;
    b.n = (z * R.ny + y) * R.nx + x;
    b.dx[0] = x == 0 ? R.nx - 1 : -1;
    b.dx[1] = x == R.nx - 1 ? -(R.nx - 1) : 1;
    b.dy[0] = (y == 0 ? R.ny - 1 : -1) * R.nx;
    b.dy[1] = (y == R.ny - 1 ? -(R.ny - 1) : 1) * R.nx;
    b.dz[0] = (z == 0 ? R.nz - 1 : -1) * nxy;
    b.dz[1] = (z == R.nz - 1 ? -(R.nz - 1) : 1) * nxy;
    b.ylo_wall = R.ywall && y == 0;
    b.yhi_wall = R.ywall && y == R.ny - 1;
    b.first = R.first != 0;
    b.sol = 0u;
    return b;
}
// Directions arriving from beyond a y wall: e_y > 0 at the low wall (sgn > 0), e_y < 0 at
// the high wall.
template <class Lat>
__host__ __device__ constexpr unsigned ymask(int sgn) {
    unsigned m = 0u;
    for (int i = 1; i < Lat::Q; ++i)
        if (sgn > 0 ? Lat::e(i, 1) > 0 : Lat::e(i, 1) < 0) m |= 1u << i;
    return m;
}
// Memory access by plane and slot through raw buffer instructions: a uniform resource
// for a group of planes (scalar registers), the plane's byte offset as the scalar offset
// and the slot's as the per-lane 32-bit offset, so that a pull holds one vector register
// for its address.  Offsets stay below 2^32 by the size limits of vlb3_create (a group
// is at most one lattice of 19 planes).
using rsrc_t = __amdgpu_buffer_rsrc_t;
using u32x2 = __attribute__((ext_vector_type(2))) unsigned;
template <class S>
struct Planes {
    rsrc_t r;
    unsigned stride;  // bytes per plane
};
template <class S>
__device__ __forceinline__ Planes<S> planes(const S* base, int N) {
    // stride 0 (raw), no range limit, the data format the untyped loads expect on gfx9
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(base), (short)0, -1, 0x00020000),
            (unsigned)N * (unsigned)sizeof(S)};
}
__device__ __forceinline__ float bload(float*, rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, 0));
}
__device__ __forceinline__ double bload(double*, rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, 0));
}
__device__ __forceinline__ void bstore(float x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, (int)v, (int)s, 0);
}
__device__ __forceinline__ void bstore(double x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, (int)v, (int)s, 0);
}
template <class S>
__device__ __forceinline__ S at(const Planes<S>& P, int plane, int slot) {
    return bload((S*)nullptr, P.r, (unsigned)slot * (unsigned)sizeof(S), (unsigned)plane * P.stride);
}
template <class S>
__device__ __forceinline__ void put(const Planes<S>& P, int plane, int slot, T v) {
    bstore((S)v, P.r, (unsigned)slot * (unsigned)sizeof(S), (unsigned)plane * P.stride);
}
// The 19 planes of lattice L of the source or destination buffer.
template <class Lat, class S>
__device__ __forceinline__ Planes<S> src_lattice(const Run3<S>& R, int L) {
    return planes(R.src + (size_t)L * Lat::Q * (size_t)R.N, R.N);
}
template <class Lat, class S>
__device__ __forceinline__ Planes<S> dst_lattice(const Run3<S>& R, int L) {
    return planes((const S*)R.dst + (size_t)L * Lat::Q * (size_t)R.N, R.N);
}
// Population i of a lattice arriving at the node from x - e_i with the periodic wrap in
// all three axes (the wall fix-up below replaces the pulls from beyond a y wall).
template <class Lat, class S>
__device__ __forceinline__ S pullb(const Planes<S>& P, const Nbr& b, int i) {
    if (b.first) return at(P, i, b.n);
    const int ex = Lat::e(i, 0), ey = Lat::e(i, 1), ez = Lat::e(i, 2);
    const int s = b.n + (ex > 0 ? b.dx[0] : (ex < 0 ? b.dx[1] : 0)) +
                  (ey > 0 ? b.dy[0] : (ey < 0 ? b.dy[1] : 0)) +
                  (ez > 0 ? b.dz[0] : (ez < 0 ? b.dz[1] : 0));
    return at(P, i, s);
}
// A copy of the pull offsets that the compiler cannot hoist out of a lattice loop (the
// empty asm redefines them), so that each iteration recomputes the 19 slots instead of
// holding them in registers across the loop.
__device__ __forceinline__ Nbr fresh(const Nbr& b) {
    Nbr c = b;
    asm volatile("" : "+v"(c.n), "+v"(c.dx[0]), "+v"(c.dx[1]), "+v"(c.dy[0]), "+v"(c.dy[1]),
                 "+v"(c.dz[0]), "+v"(c.dz[1]));
    return c;
}
// Pulls of lattice L with the directions arriving from beyond a y wall or from a solid
// node taken as the node's own post-collision value of the opposite direction.  (A wave
// holds one row, so the wall branches are uniform.)
template <class Lat, class S>
__device__ __forceinline__ void pull_all(const Run3<S>& R, const Nbr& b, int L, S g[Lat::Q]) {
    const Planes<S> P = src_lattice<Lat>(R, L);
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) g[i] = pullb<Lat>(P, b, i);
    if (b.first) return;
    if (b.ylo_wall) {
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i)
            if (Lat::e(i, 1) > 0) g[i] = at(P, opp(i), b.n);
    }
    if (b.yhi_wall) {
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i)
            if (Lat::e(i, 1) < 0) g[i] = at(P, opp(i), b.n);
    }
    if (b.sol) {
#pragma unroll
        for (int i = 1; i < Lat::Q; ++i)
            if ((b.sol >> i) & 1u) g[i] = at(P, opp(i), b.n);
    }
}

template <class Lat, class S>
__device__ __forceinline__ void hydro_pull(const Run3<S>& R, const Nbr& b, S f[Lat::Q], T& rho, T u[3]) {
    pull_all<Lat>(R, b, 0, f);
    T dr = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
        const T v = (T)f[i];
        dr += v;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (Lat::e(i, a) != 0) j[a] += Lat::e(i, a) > 0 ? v : -v;
    }
    rho = 1.0 + dr;
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * R.F[a]) / rho;
}

#ifndef VLB3_XCD_ROWS
#define VLB3_XCD_ROWS 1
#endif
// Tile of this block (x tile, y tile, z).  With VLB3_XCD_ROWS (the default) the x tiles
// of one tile row (a y tile and z) run on one XCD -- the hardware deals consecutive
// blocks to the eight XCDs in turn -- so that the cache lines two x-neighbouring tiles
// share (the pulls shifted by one node in x) come into one L2 once; rows beyond the
// last multiple of eight keep the plain order.  On the 256 x 64 x 256 channel this cuts
// the step kernel's HBM reads from 1.29x to 1.03x of the algorithmic bytes (D3Q19).
__device__ __forceinline__ void tile_of(int& bx, int& by, int& bz) {
    if (VLB3_XCD_ROWS) {
        const int nxt = gridDim.x, nyt = gridDim.y, rows = nyt * gridDim.z;
        const int b = blockIdx.x + nxt * (blockIdx.y + nyt * blockIdx.z);
        int row, xt;
        if (b < nxt * (rows & ~7)) {
            const int s = b >> 3;
            row = 8 * (s / nxt) + (b & 7);
            xt = s - (s / nxt) * nxt;
        } else {
            row = b / nxt;
            xt = b - row * nxt;
        }
        bx = xt;
        by = row % nyt;
        bz = row / nyt;
    } else {
        bx = blockIdx.x;
        by = blockIdx.y;
        bz = blockIdx.z;
    }
}

template <class S, class Lat, bool SOLIDS>
__global__ __launch_bounds__(TX * TY) void k3_macro(Run3<S> R) {
    int bx, by, z;
    tile_of(bx, by, z);
    const int x = bx * TX + threadIdx.x, y = by * TY + threadIdx.y;
    if (x >= R.nx || y >= R.ny) return;
    Nbr b = make_nbr(R, x, y, z);
    const int n = b.n;
    if (SOLIDS) {
        const unsigned bits = R.bits[n];
        if (bits & SELF_SOLID) return;
        b.sol = bits & ~SELF_SOLID;
    }
    S f[Lat::Q];
    T rho, u[3];
    hydro_pull<Lat>(R, b, f, rho, u);
    const Planes<S> M = planes((const S*)R.mac, R.N);
    put(M, 0, n, rho);
#pragma unroll
    for (int a = 0; a < 3; ++a) put(M, 1 + a, n, u[a]);
}

// Derivative along one axis: central difference, or next to a flat half-way wall the
// quadratic through the no-slip value half a spacing away.
__device__ __forceinline__ T fd(bool lo_wall, T vlo, T v0, bool hi_wall, T vhi) {
    if (!lo_wall && !hi_wall) return 0.5 * (vhi - vlo);
    if (lo_wall && !hi_wall) return (1.0 / 3.0) * vhi + v0;
    if (!lo_wall) return -((1.0 / 3.0) * vlo + v0);
    return 0.0;
}

// Collision of conformation lattice k (a run-time index, so that the six lattices share
// one copy of the code and its registers) from its pulled populations: CNEBB at a
// wall-adjacent node, moments, collision, store.
__device__ __forceinline__ T phi0_rt(int k) { return (k == 0 || k == 3 || k == 5) ? 1.0 : 0.0; }
// BOTH: an unknown's opposite may be unknown too (solid nodes on both sides of a lattice
// line); never next to the flat y walls alone.
template <class Lat, bool BOTH, class S>
__device__ __forceinline__ void conf_collide(const Run3<S>& R, int n, int k, const S gs[Lat::Q], const T u[3],
                                             const T up[3], T rho, T uu, T dp, T Sk, T Spk,
                                             unsigned unk) {
    const T phi = phi0_rt(k) + dp;
    // first and second moments of the pulled deviations
    T J[3] = {0.0, 0.0, 0.0}, P[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
        const T v = (T)gs[i];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (Lat::e(i, a) != 0) J[a] += Lat::e(i, a) > 0 ? v : -v;
#pragma unroll
        for (int m = 0; m < 6; ++m)
            if (Lat::e(i, ka(m)) * Lat::e(i, kb(m)) != 0) P[m] += (Lat::e(i, ka(m)) * Lat::e(i, kb(m)) > 0) ? v : -v;
    }
    if (unk) {
        // CNEBB: each unknown (a direction arriving from beyond a wall or from a solid
        // node) becomes the
        // equilibrium deviation at (phi_b, u_b) plus the non-equilibrium part of its known
        // opposite; g_0 takes the remainder of phi_b, so the zeroth moment is unchanged
        // and the first and second moments change by the unknowns' corrections only.
#pragma unroll
        for (int i = 1; i < Lat::Q; ++i) {
            if ((unk >> i) & 1u) {
                const int o = opp(i);
                const T eui = Lat::e(i, 0) * u[0] + Lat::e(i, 1) * u[1] + Lat::e(i, 2) * u[2];
                const T eqi = Lat::w(i) * (dp + phi * (3.0 * eui + 4.5 * (eui * eui - CS2 * uu)));
                const T eqo = Lat::w(o) * (dp + phi * (-3.0 * eui + 4.5 * (eui * eui - CS2 * uu)));
                // (an unknown whose opposite is unknown too: the equilibrium alone)
                const T delta = (BOTH && ((unk >> o) & 1u)) ? eqi - (T)gs[i]
                                                            : eqi + (T)gs[o] - eqo - (T)gs[i];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (Lat::e(i, a) != 0) J[a] += Lat::e(i, a) > 0 ? delta : -delta;
#pragma unroll
                for (int m = 0; m < 6; ++m)
                    if (Lat::e(i, ka(m)) * Lat::e(i, kb(m)) != 0)
                        P[m] += (Lat::e(i, ka(m)) * Lat::e(i, kb(m)) > 0) ? delta : -delta;
            }
        }
    }
    // B1 = J - phi u; B2 = P - c_s^2 d (phi - phi0) - phi u u (deviations carry phi0)
    T B1[3], B2[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) B1[a] = J[a] - phi * u[a];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int a = ka(m), b = kb(m);
        B2[m] = P[m] - (a == b ? CS2 * dp : 0.0) - phi * u[a] * u[b];
    }
    const T trB2 = B2[0] + B2[3] + B2[5];
    // Post-collision deviation g_i - w_i phi0 = w_i (c0 + e_i.c + e_i.M.e_i), collecting
    // the equilibrium phi (1 + 3 e.u + 4.5 ((e.u)^2 - c_s^2 u.u)), the regularized
    // non-equilibrium p1 3 e.B1 + p2 4.5 (e.B2.e - c_s^2 tr B2), the auxiliary term
    // 3 h2 (e.F) phi / rho and the source term 1.5 F~(t) - 0.5 F~(t-1) with
    // F~ = S (1 + 3 h2 e.u):
    T c0 = dp - 1.5 * phi * uu - 1.5 * R.p2 * trB2 + 1.5 * Sk - 0.5 * Spk;
    T c[3], M[6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        c[a] = 3.0 * phi * u[a] + 3.0 * R.p1 * B1[a] + 3.0 * R.h2 * R.F[a] * phi / rho +
               3.0 * R.h2 * (1.5 * Sk * u[a] - 0.5 * Spk * up[a]);
#pragma unroll
    for (int m = 0; m < 6; ++m) M[m] = 4.5 * (phi * u[ka(m)] * u[kb(m)] + R.p2 * B2[m]);
    const Planes<S> out = dst_lattice<Lat>(R, 1 + k);
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) put(out, i, n, Lat::w(i) * quad_at<Lat>(i, c0, c, M));
}

// Pulls and collision of conformation lattice k.
template <class Lat, bool BOTH, class S>
__device__ __forceinline__ void conf_lattice(const Run3<S>& R, const Nbr& nb, int k, const T u[3],
                                             const T up[3], T rho, T uu, T dp, T Sk, T Spk,
                                             unsigned unk) {
    const Nbr b = fresh(nb);
    S gs[Lat::Q];
    pull_all<Lat>(R, b, 1 + k, gs);
    conf_collide<Lat, BOTH>(R, b.n, k, gs, u, up, rho, uu, dp, Sk, Spk, unk);
}

// WALLS: the y walls' fix-ups, one-sided differences and CNEBB compiled in (a wave holds
// one row, so they are uniform branches); without walls they are compiled out.
// SOLIDS: solid nodes present (their own lanes idle; their faces act as half-way walls).
// CLOSURE: a constitutive closure other than Oldroyd-B (compiled apart, so that the
// Oldroyd-B kernels keep their registers).
template <class S, class Lat, bool WALLS, bool SOLIDS, int HOLD, bool CLOSURE>
__global__ __launch_bounds__(TX * TY) void k3_step(Run3<S> R) {
    int bx, by, z;
    tile_of(bx, by, z);
    const int x = bx * TX + threadIdx.x, y = by * TY + threadIdx.y;
    if (x >= R.nx || y >= R.ny) return;
    const long long N = R.N;
    Nbr nbr = make_nbr(R, x, y, z);
    if (!WALLS) nbr.ylo_wall = nbr.yhi_wall = false;
    const int n = nbr.n;
    if (SOLIDS) {
        const unsigned bits = R.bits[n];
        if (bits & SELF_SOLID) return;
        nbr.sol = bits & ~SELF_SOLID;
    }

    // ---- hydrodynamic pulls, rho, u ----
    S f[Lat::Q];
    T rho, u[3];
    hydro_pull<Lat>(R, nbr, f, rho, u);

    // ---- conformation (zeroth moments of the pulled populations; CNEBB keeps them) ----
    // Per-lattice values wait in LDS, one column per lane, so that the lattice loops run
    // with a run-time index and one lattice's registers.
    __shared__ T s_dphi[6][TX * TY], s_Sc[6][TX * TY], s_Sp[6][TX * TY];
    const int tid = threadIdx.y * TX + threadIdx.x;
    T dphi[6];
    S G[HOLD > 0 ? HOLD : 1][Lat::Q];  // the held lattices 6 - HOLD .. 5
#pragma unroll 1
    for (int k = 0; k < 6 - HOLD; ++k) {
        S g[Lat::Q];
        pull_all<Lat>(R, fresh(nbr), 1 + k, g);
        T s = 0.0;
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i) s += (T)g[i];
        s_dphi[k][tid] = s;
    }
#pragma unroll
    for (int j = 0; j < HOLD; ++j) {
        const int k = 6 - HOLD + j;
        pull_all<Lat>(R, nbr, 1 + k, G[j]);
        T s = 0.0;
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i) s += (T)G[j][i];
        s_dphi[k][tid] = s;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) dphi[k] = s_dphi[k][tid];

    // ---- velocity gradient L[g][b] = d_g u_b and D_a = d_a(rho u_a^3) at time n ----
    T L[3][3], D[3];
    {
        const Planes<S> mac = planes((const S*)R.mac, R.N);
        const bool wl = nbr.ylo_wall, wh = nbr.yhi_wall;
        const int nb[3][2] = {{n + nbr.dx[0], n + nbr.dx[1]},
                              {n + nbr.dy[0], n + nbr.dy[1]},
                              {n + nbr.dz[0], n + nbr.dz[1]}};
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            // a wall or a solid neighbour along the axis (directions 1 + 2g and 2 + 2g
            // pull from the low and the high neighbour)
            const bool lw = (g == 1 && wl) || ((nbr.sol >> (1 + 2 * g)) & 1u);
            const bool hw = (g == 1 && wh) || ((nbr.sol >> (2 + 2 * g)) & 1u);
            T rl = 0.0, rh = 0.0, vl[3] = {0.0, 0.0, 0.0}, vh[3] = {0.0, 0.0, 0.0};
            if (!lw) {
                rl = at(mac, 0, nb[g][0]);
#pragma unroll
                for (int b = 0; b < 3; ++b) vl[b] = at(mac, 1 + b, nb[g][0]);
            }
            if (!hw) {
                rh = at(mac, 0, nb[g][1]);
#pragma unroll
                for (int b = 0; b < 3; ++b) vh[b] = at(mac, 1 + b, nb[g][1]);
            }
#pragma unroll
            for (int b = 0; b < 3; ++b) L[g][b] = fd(lw, vl[b], u[b], hw, vh[b]);
            D[g] = fd(lw, rl * vl[g] * vl[g] * vl[g], rho * u[g] * u[g] * u[g], hw,
                      rh * vh[g] * vh[g] * vh[g]);
        }
    }

    // ---- constitutive source and polymer stress of the closure (B = A - I = dphi) ----
    T Sc[6], tau[6];
    {
        T A[3][3];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            A[ka(k)][kb(k)] = phi0(k) + dphi[k];
            A[kb(k)][ka(k)] = phi0(k) + dphi[k];
        }
        // relaxation function F_r and stress function F_s (Oldroyd-B: both B)
        T Fr[6], Fs[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) Fr[k] = Fs[k] = dphi[k];
        const T trB = dphi[0] + dphi[3] + dphi[5];
        if (!CLOSURE) {
        } else if (R.model == VLB_GIESEKUS) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int a = ka(k), b = kb(k);
                T bb = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) bb += (A[a][c] - (a == c ? 1.0 : 0.0)) * (A[c][b] - (c == b ? 1.0 : 0.0));
                Fr[k] += R.mpar * bb;
            }
        } else if (R.model == VLB_LPTT || R.model == VLB_EPTT) {
            const T Y = R.model == VLB_LPTT ? 1.0 + R.mpar * trB : exp(R.mpar * trB);
#pragma unroll
            for (int k = 0; k < 6; ++k) Fr[k] = Y * dphi[k];
        } else if (R.model == VLB_FENE_P) {
            const T f = (R.mpar - 3.0) / (R.mpar - 3.0 - trB);  // (L^2 - 3) / (L^2 - tr A)
#pragma unroll
            for (int k = 0; k < 6; ++k) Fr[k] = Fs[k] = f * (phi0(k) + dphi[k]) - phi0(k);
        }
        const T trL = L[0][0] + L[1][1] + L[2][2];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int a = ka(k), b = kb(k);
            T s = -R.inv_lam * Fr[k];
#pragma unroll
            for (int g = 0; g < 3; ++g) s += A[a][g] * L[g][b] + A[g][b] * L[g][a];
            s += A[a][b] * trL;
            Sc[k] = R.no_source ? 0.0 : s;
            tau[k] = R.eta_over_lam * Fs[k];
        }
    }
    // history: S and u of the previous step (the first step takes this step's)
    const Planes<S> hist = planes((const S*)R.hist, R.N);
    T up[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        s_Sc[k][tid] = Sc[k];
        s_Sp[k][tid] = R.first ? Sc[k] : (T)at(hist, k, n);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) up[a] = R.first ? u[a] : (T)at(hist, 6 + a, n);

    // ---- hydrodynamic collision (moment form) ----
    {
        const Planes<S> out = dst_lattice<Lat>(R, 0);
        // second moments and third-order basis moments of the pulled deviations
        T P[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, Qm[Lat::NB3];
#pragma unroll
        for (int m = 0; m < Lat::NB3; ++m) Qm[m] = 0.0;
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i) {
            const T v = (T)f[i];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if (Lat::e(i, ka(k)) * Lat::e(i, kb(k)) != 0) P[k] += (Lat::e(i, ka(k)) * Lat::e(i, kb(k)) > 0) ? v : -v;
#pragma unroll
            for (int m = 0; m < Lat::NB3; ++m)
                if (Lat::h3(i, m) != 0.0) Qm[m] += Lat::h3(i, m) * v;
        }
        // off-equilibrium moments: A1 = -F/2 (literal), A2 = Pi - c_s^2 d (rho - 1) - rho u u
        // (deviations carry the rest part), A3 along each basis function: moment - rho u3
        const T dr = rho - 1.0;
        T A2[6], A3[Lat::NB3], uc[Lat::NB3];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int a = ka(k), b = kb(k);
            A2[k] = P[k] - (a == b ? CS2 * dr : 0.0) - rho * u[a] * u[b];
        }
#pragma unroll
        for (int m = 0; m < Lat::NB3; ++m) {
            uc[m] = Lat::u3(m, u);
            A3[m] = Qm[m] - rho * uc[m];
        }
        const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const T trA2 = A2[0] + A2[3] + A2[5], trt = tau[0] + tau[3] + tau[5];
        // Post-collision deviation f_i - w_i = w_i (c0 + e_i.c + e_i.M.e_i + sum_m h_m(e_i)
        // d_m), collecting the equilibrium, c1 times the regularized orders 1-2 (A1 =
        // -F/2), c2 times the projected third order, G_i, T_i and F_i:
        const T c0 = dr - 1.5 * rho * uu - 1.5 * R.c1 * trA2 +
                     1.5 * R.h1 * (D[0] + D[1] + D[2]) + 1.5 * R.inv_ts1 * trt;
        T c[3], M[6], d[Lat::NB3];
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] = 3.0 * rho * u[a] - 1.5 * R.c1 * R.F[a] + 3.0 * R.h1 * R.F[a];
#pragma unroll
        for (int m = 0; m < 6; ++m)
            M[m] = 4.5 * (rho * u[ka(m)] * u[kb(m)] + R.c1 * A2[m] - R.inv_ts1 * tau[m]);
        M[0] -= 4.5 * R.h1 * D[0];
        M[3] -= 4.5 * R.h1 * D[1];
        M[5] -= 4.5 * R.h1 * D[2];
#pragma unroll
        for (int m = 0; m < Lat::NB3; ++m) d[m] = Lat::h3inv(m) * (rho * uc[m] + R.c2 * A3[m]);
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i) {
            T v = quad_at<Lat>(i, c0, c, M);
#pragma unroll
            for (int m = 0; m < Lat::NB3; ++m)
                if (Lat::h3(i, m) != 0.0) v += Lat::h3(i, m) * d[m];
            put(out, i, n, Lat::w(i) * v);
        }
    }

    // ---- conformation lattices: pulls, CNEBB at wall-adjacent nodes, collision ----
    // directions CNEBB rebuilds (none on the first step: its pulls are the node's own slots)
    const unsigned unk = R.first ? 0u
                                 : ((WALLS && nbr.ylo_wall) ? ymask<Lat>(1) : 0u) |
                                       ((WALLS && nbr.yhi_wall) ? ymask<Lat>(-1) : 0u) | nbr.sol;
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    // The held lattices (the last HOLD of the zeroth-moment pass) from their registers,
    // then the others pulled again, most recently read first.
#pragma unroll
    for (int j = HOLD - 1; j >= 0; --j) {
        const int k = 6 - HOLD + j;
        // (held in storage precision: the empty asm keeps the widened copies of the
        // zeroth-moment sum from being kept instead)
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i) asm volatile("" : "+v"(G[j][i]));
        conf_collide<Lat, SOLIDS>(R, n, k, G[j], u, up, rho, uu, s_dphi[k][tid], s_Sc[k][tid], s_Sp[k][tid],
                     unk);
    }
#pragma unroll 1
    for (int k = 5 - HOLD; k >= 0; --k)
        conf_lattice<Lat, SOLIDS>(R, nbr, k, u, up, rho, uu, s_dphi[k][tid], s_Sc[k][tid], s_Sp[k][tid], unk);
#pragma unroll
    for (int k = 0; k < 6; ++k) put(hist, k, n, s_Sc[k][tid]);
#pragma unroll
    for (int a = 0; a < 3; ++a) put(hist, 6 + a, n, u[a]);
}

// Equilibrium state of the given fields at every node's own slot (read without a pull
// by the first step); history cleared.
template <class S, class Lat>
__global__ __launch_bounds__(TX * TY) void k3_init(Run3<S> R, S* pop, const S* const* fields) {
    const int x = blockIdx.x * TX + threadIdx.x, y = blockIdx.y * TY + threadIdx.y, z = blockIdx.z;
    if (x >= R.nx || y >= R.ny) return;
    const long long N = R.N;
    const int n = (z * R.ny + y) * R.nx + x;
    T v[10];
    const T dflt[10] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 1.0};
#pragma unroll
    for (int c = 0; c < 10; ++c) v[c] = fields[c] ? (T)fields[c][n] : dflt[c];
    const T rho = v[0], u[3] = {v[1], v[2], v[3]};
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T uc[Lat::NB3];
#pragma unroll
    for (int m = 0; m < Lat::NB3; ++m) uc[m] = Lat::u3(m, u);
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
        const T eu = Lat::e(i, 0) * u[0] + Lat::e(i, 1) * u[1] + Lat::e(i, 2) * u[2];
        T third = 0.0;
#pragma unroll
        for (int m = 0; m < Lat::NB3; ++m) third += Lat::h3inv(m) * Lat::h3(i, m) * uc[m];
        pop[(long long)i * N + n] = (S)(Lat::w(i) * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * (eu * eu - CS2 * uu) + third)));
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const T phi = v[4 + k];
            pop[((long long)(1 + k) * Lat::Q + i) * N + n] =
                (S)(Lat::w(i) * ((phi - phi0(k)) + phi * (3.0 * eu + 4.5 * (eu * eu - CS2 * uu))));
        }
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) R.hist[c * N + n] = (S)0.0;
}

// rho, u (half-force shift) and A of the current state.
template <class S, class Lat>
__global__ __launch_bounds__(TX * TY) void k3_read(Run3<S> R, S* const* out) {
    const int x = blockIdx.x * TX + threadIdx.x, y = blockIdx.y * TY + threadIdx.y, z = blockIdx.z;
    if (x >= R.nx || y >= R.ny) return;
    Nbr nbr = make_nbr(R, x, y, z);
    const int n = nbr.n;
    if (R.bits) {
        const unsigned bits = R.bits[n];
        if (bits & SELF_SOLID) {  // solid node: read out at rest
            const T rest[10] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 1.0};
#pragma unroll
            for (int c = 0; c < 10; ++c)
                if (out[c]) out[c][n] = (S)rest[c];
            return;
        }
        nbr.sol = bits & ~SELF_SOLID;
    }
    S f[Lat::Q];
    T rho, u[3];
    hydro_pull<Lat>(R, nbr, f, rho, u);
    T v[10] = {rho, u[0], u[1], u[2]};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        S g[Lat::Q];
        pull_all<Lat>(R, nbr, 1 + k, g);
        T s = 0.0;
#pragma unroll
        for (int i = 0; i < Lat::Q; ++i) s += (T)g[i];
        v[4 + k] = phi0(k) + s;
    }
#pragma unroll
    for (int c = 0; c < 10; ++c)
        if (out[c]) out[c][n] = (S)v[c];
}

}  // namespace
}  // namespace vlb3

// ---------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------
struct vlb3_sim {
    int nx, ny, nz, q, prec, ywall;
    size_t esz;
    long long N, P;  // nodes; plane stride in elements
    bool bound = false, params_set = false, inited = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    size_t off_pop[2] = {0, 0}, off_hist = 0, off_mac = 0, off_bits = 0, off_ptrs = 0, total = 0;
    bool has_solid = false;  // a solid mask is set (the bits plane in the workspace)
    int parity = 0, first = 1;
    int64_t step = 0;
    double nu_s = 0, eta_p = 0, lam = 1, kappa = 0, Ls = 0.25, Lp = 1e-6, F[3] = {0, 0, 0};
    int flags = 0;
    int model = VLB_OLDROYD_B;
    double mpar = 0.0;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
// Plane stride: the node count rounded up to 64 elements plus 4160 (4096 + 64), so that
// the 133 (189) planes a node touches do not all start at the same offset modulo a large
// power of two (worth about 4% on a 2^22-node grid).
long long plane_stride(long long N) { return ((N + 63) & ~63LL) + 4160; }

void layout(vlb3_sim* s) {
    size_t o = 0;
    auto take = [&](size_t b) { const size_t r = o; o = align256(o + b); return r; };
    const size_t plane = (size_t)s->P * s->esz;
    s->off_pop[0] = take((size_t)vlb3::NLAT * s->q * plane);
    s->off_pop[1] = take((size_t)vlb3::NLAT * s->q * plane);
    s->off_hist = take(9 * plane);
    s->off_mac = take(4 * plane);
    s->off_bits = take((size_t)s->P * sizeof(unsigned));
    s->off_ptrs = take(10 * sizeof(void*));
    s->total = o;
}

template <class S>
vlb3::Run3<S> make_run(const vlb3_sim* s) {
    vlb3::Run3<S> r{};
    r.nx = s->nx;
    r.ny = s->ny;
    r.nz = s->nz;
    r.ywall = s->ywall;
    r.first = s->first;
    r.N = (int)s->P;
    r.src = reinterpret_cast<const S*>(s->ws + s->off_pop[s->parity]);
    r.dst = reinterpret_cast<S*>(s->ws + s->off_pop[s->parity ^ 1]);
    r.hist = reinterpret_cast<S*>(s->ws + s->off_hist);
    r.mac = reinterpret_cast<S*>(s->ws + s->off_mac);
    r.bits = s->has_solid ? reinterpret_cast<const unsigned*>(s->ws + s->off_bits) : nullptr;
    // relaxation times from the transport coefficients (Sec. 3.1-3.2), c_s^2 = 1/3
    const double ts1 = 3.0 * s->nu_s + 0.5, ts2 = s->Ls / (3.0 * s->nu_s) + 0.5;
    const double tp1 = 3.0 * s->kappa + 0.5, tp2 = s->Lp / (3.0 * s->kappa) + 0.5;
    r.c1 = 1.0 - 1.0 / ts1;
    r.c2 = 1.0 - 1.0 / ts2;
    r.h1 = 1.0 - 1.0 / (2.0 * ts1);
    r.inv_ts1 = 1.0 / ts1;
    r.p1 = 1.0 - 1.0 / tp1;
    r.p2 = 1.0 - 1.0 / tp2;
    r.h2 = 1.0 - 1.0 / (2.0 * tp1);
    r.inv_lam = 1.0 / s->lam;
    r.eta_over_lam = s->eta_p / s->lam;
    for (int a = 0; a < 3; ++a) r.F[a] = s->F[a];
    r.no_source = (s->flags & VLB_FLAG_NO_SOURCE) ? 1 : 0;
    r.model = s->model;
    r.mpar = s->mpar;
    return r;
}

dim3 grid_of(const vlb3_sim* s) {
    return dim3((unsigned)((s->nx + vlb3::TX - 1) / vlb3::TX),
                (unsigned)((s->ny + vlb3::TY - 1) / vlb3::TY), (unsigned)s->nz);
}

int check_ready(const vlb3_sim* s) {
    if (!s) return vlb::report_error(VLB_E_INVALID_ARG, "null simulation");
    if (!s->bound) return vlb::report_error(VLB_E_STATE, "workspace not bound (vlb3_bind)");
    if (!s->params_set) return vlb::report_error(VLB_E_STATE, "parameters not set (vlb3_set_params)");
    return VLB_OK;
}

#define VLB3_HIP(expr)                                                                           \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return vlb::report_error(VLB_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class S, class Lat>
int do_steps(vlb3_sim* s, int64_t n) {
    const dim3 blk(vlb3::TX, vlb3::TY), grd = grid_of(s);
    constexpr int hold = vlb3::kHold<S, Lat>;
    for (int64_t k = 0; k < n; ++k) {
        const vlb3::Run3<S> r = make_run<S>(s);
        if (s->has_solid) {  // (the wall code is compiled in; it checks the y walls itself)
            hipLaunchKernelGGL((vlb3::k3_macro<S, Lat, true>), grd, blk, 0, s->stream, r);
            if (s->model != VLB_OLDROYD_B)
                hipLaunchKernelGGL((vlb3::k3_step<S, Lat, true, true, vlb3::kHold<S, Lat, true, true>, true>), grd, blk, 0, s->stream, r);
            else
                hipLaunchKernelGGL((vlb3::k3_step<S, Lat, true, true, vlb3::kHold<S, Lat, true>, false>), grd, blk, 0, s->stream, r);
        } else {
            hipLaunchKernelGGL((vlb3::k3_macro<S, Lat, false>), grd, blk, 0, s->stream, r);
            if (s->model != VLB_OLDROYD_B) {
                constexpr int hc = vlb3::kHold<S, Lat, false, true>;
                if (s->ywall)
                    hipLaunchKernelGGL((vlb3::k3_step<S, Lat, true, false, hc, true>), grd, blk, 0, s->stream, r);
                else
                    hipLaunchKernelGGL((vlb3::k3_step<S, Lat, false, false, hc, true>), grd, blk, 0, s->stream, r);
            } else if (s->ywall) {
                hipLaunchKernelGGL((vlb3::k3_step<S, Lat, true, false, hold, false>), grd, blk, 0, s->stream, r);
            } else {
                hipLaunchKernelGGL((vlb3::k3_step<S, Lat, false, false, hold, false>), grd, blk, 0, s->stream, r);
            }
        }
        VLB3_HIP(hipGetLastError());
        s->parity ^= 1;
        s->first = 0;
        ++s->step;
    }
    return VLB_OK;
}

template <class S, class Lat>
int do_init(vlb3_sim* s, const void* const fields[10]) {
    void* host_ptrs[10];
    for (int c = 0; c < 10; ++c) host_ptrs[c] = const_cast<void*>(fields ? fields[c] : nullptr);
    void** dev_ptrs = reinterpret_cast<void**>(s->ws + s->off_ptrs);
    VLB3_HIP(hipMemcpyAsync(dev_ptrs, host_ptrs, sizeof(host_ptrs), hipMemcpyHostToDevice, s->stream));
    s->parity = 0;
    s->first = 1;
    s->step = 0;
    const vlb3::Run3<S> r = make_run<S>(s);
    hipLaunchKernelGGL((vlb3::k3_init<S, Lat>), grid_of(s), dim3(vlb3::TX, vlb3::TY), 0, s->stream, r,
                       reinterpret_cast<S*>(s->ws + s->off_pop[0]),
                       reinterpret_cast<const S* const*>(dev_ptrs));
    VLB3_HIP(hipGetLastError());
    // the pointer table is read by the kernel: keep the host copy alive until it ran
    VLB3_HIP(hipStreamSynchronize(s->stream));
    s->inited = true;
    return VLB_OK;
}

template <class S, class Lat>
int do_read(vlb3_sim* s, void* const out[10]) {
    void* host_ptrs[10];
    for (int c = 0; c < 10; ++c) host_ptrs[c] = out ? out[c] : nullptr;
    void** dev_ptrs = reinterpret_cast<void**>(s->ws + s->off_ptrs);
    VLB3_HIP(hipMemcpyAsync(dev_ptrs, host_ptrs, sizeof(host_ptrs), hipMemcpyHostToDevice, s->stream));
    const vlb3::Run3<S> r = make_run<S>(s);
    hipLaunchKernelGGL((vlb3::k3_read<S, Lat>), grid_of(s), dim3(vlb3::TX, vlb3::TY), 0, s->stream, r,
                       reinterpret_cast<S* const*>(dev_ptrs));
    VLB3_HIP(hipGetLastError());
    VLB3_HIP(hipStreamSynchronize(s->stream));
    return VLB_OK;
}

}  // namespace

// FP64 entry points (defined in the VLB3_PART 2 translation unit).
namespace vlb3_f64 {
int steps(vlb3_sim* s, int64_t n);
int init(vlb3_sim* s, const void* const* fields);
int read(vlb3_sim* s, void* const* out);
}  // namespace vlb3_f64

#if VLB3_PART == 2
namespace vlb3_f64 {
int steps(vlb3_sim* s, int64_t n) {
    return s->q == 27 ? do_steps<double, vlb3::D3Q27>(s, n) : do_steps<double, vlb3::D3Q19>(s, n);
}
int init(vlb3_sim* s, const void* const* f) {
    return s->q == 27 ? do_init<double, vlb3::D3Q27>(s, f) : do_init<double, vlb3::D3Q19>(s, f);
}
int read(vlb3_sim* s, void* const* o) {
    return s->q == 27 ? do_read<double, vlb3::D3Q27>(s, o) : do_read<double, vlb3::D3Q19>(s, o);
}
}  // namespace vlb3_f64
#else
namespace {

// Entry points by storage type and lattice.
template <class Lat>
struct StepOp {
    static int run(vlb3_sim* s, int64_t n) { return do_steps<float, Lat>(s, n); }
    static int f64(vlb3_sim* s, int64_t n) { return vlb3_f64::steps(s, n); }
};
template <class Lat>
struct InitOp {
    static int run(vlb3_sim* s, const void* const* f) { return do_init<float, Lat>(s, f); }
    static int f64(vlb3_sim* s, const void* const* f) { return vlb3_f64::init(s, f); }
};
template <class Lat>
struct ReadOp {
    static int run(vlb3_sim* s, void* const* o) { return do_read<float, Lat>(s, o); }
    static int f64(vlb3_sim* s, void* const* o) { return vlb3_f64::read(s, o); }
};
template <template <class> class Op, class Arg>
int by_kind(vlb3_sim* s, Arg a) {
    if (s->prec == VLB_FP32) return s->q == 27 ? Op<vlb3::D3Q27>::run(s, a) : Op<vlb3::D3Q19>::run(s, a);
    return Op<vlb3::D3Q19>::f64(s, a);
}

}  // namespace

extern "C" {

int vlb3_create(int nx, int ny, int nz, int q, int prec, int ymode, vlb3_sim** out) {
    if (!out) return vlb::report_error(VLB_E_INVALID_ARG, "null output");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return vlb::report_error(VLB_E_INVALID_ARG, "grid sizes must be >= 1");
    if (q != 19 && q != 27) return vlb::report_error(VLB_E_INVALID_ARG, "lattice must be 19 (D3Q19) or 27 (D3Q27)");
    if (prec != VLB_FP32 && prec != VLB_FP64) return vlb::report_error(VLB_E_INVALID_ARG, "unknown precision");
    if (ymode != VLB_PERIODIC && ymode != VLB_WALL)
        return vlb::report_error(VLB_E_INVALID_ARG, "ymode must be VLB_PERIODIC or VLB_WALL");
    if (ymode == VLB_WALL && ny < 3) return vlb::report_error(VLB_E_INVALID_ARG, "walls need ny >= 3");
    if (nz > 65535 || (ny + vlb3::TY - 1) / vlb3::TY > 65535)
        return vlb::report_error(VLB_E_INVALID_ARG, "nz and the rows of blocks in y must stay within the launch grid (65535)");
    const long long N = (long long)nx * ny * nz;
    if (plane_stride(N) >= (1LL << 31) / (vlb3::NLAT * q))
        return vlb::report_error(VLB_E_INVALID_ARG, "grid too large for 32-bit plane offsets");
    vlb3_sim* s = new (std::nothrow) vlb3_sim();
    if (!s) return vlb::report_error(VLB_E_INVALID_ARG, "out of host memory");
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->q = q;
    s->prec = prec;
    s->ywall = ymode == VLB_WALL ? 1 : 0;
    s->esz = prec == VLB_FP32 ? 4 : 8;
    s->N = N;
    s->P = plane_stride(N);
    layout(s);
    *out = s;
    return VLB_OK;
}

int vlb3_set_solid(vlb3_sim* s, const unsigned char* mask) {
    if (!s) return vlb::report_error(VLB_E_INVALID_ARG, "null simulation");
    if (!s->bound) return vlb::report_error(VLB_E_STATE, "workspace not bound (vlb3_bind)");
    if (!mask) {
        s->has_solid = false;
        s->inited = false;
        return VLB_OK;
    }
    // bit i of a node: its pull in direction i comes from a solid node (x - e_i, periodic
    // in x and z, in y unless beyond a wall, which the wall rule covers); bit 31: solid
    std::vector<unsigned> bits((size_t)s->N, 0u);
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    auto ex = [&](int i, int a) { return s->q == 27 ? vlb3::D3Q27::e(i, a) : vlb3::D3Q19::e(i, a); };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = ((size_t)z * ny + y) * nx + x;
                unsigned b = mask[n] ? vlb3::SELF_SOLID : 0u;
                for (int i = 1; i < s->q; ++i) {
                    int ys = y - ex(i, 1);
                    if (ys < 0 || ys >= ny) {
                        if (s->ywall) continue;
                        ys = (ys + ny) % ny;
                    }
                    const int xs = ((x - ex(i, 0)) % nx + nx) % nx, zs = ((z - ex(i, 2)) % nz + nz) % nz;
                    if (mask[((size_t)zs * ny + ys) * nx + xs]) b |= 1u << i;
                }
                bits[n] = b;
            }
    VLB3_HIP(hipMemcpyAsync(s->ws + s->off_bits, bits.data(), bits.size() * sizeof(unsigned),
                            hipMemcpyHostToDevice, s->stream));
    VLB3_HIP(hipStreamSynchronize(s->stream));
    s->has_solid = true;
    s->inited = false;
    return VLB_OK;
}

int vlb3_set_closure(vlb3_sim* s, int model, double model_param) {
    if (!s) return vlb::report_error(VLB_E_INVALID_ARG, "null simulation");
    if (model < VLB_OLDROYD_B || model > VLB_FENE_P || !std::isfinite(model_param))
        return vlb::report_error(VLB_E_INVALID_ARG, "unknown closure or non-finite parameter");
    if (model == VLB_GIESEKUS && !(model_param >= 0.0 && model_param <= 1.0))
        return vlb::report_error(VLB_E_INVALID_ARG, "Giesekus alpha must lie in [0, 1]");
    if ((model == VLB_LPTT || model == VLB_EPTT) && !(model_param >= 0.0))
        return vlb::report_error(VLB_E_INVALID_ARG, "PTT epsilon must be >= 0");
    if (model == VLB_FENE_P && !(model_param > 3.0))
        return vlb::report_error(VLB_E_INVALID_ARG, "FENE-P needs L^2 > 3 in three dimensions");
    s->model = model;
    s->mpar = model == VLB_OLDROYD_B ? 0.0 : model_param;
    return VLB_OK;
}

int vlb3_workspace_bytes(const vlb3_sim* s, size_t* bytes) {
    if (!s || !bytes) return vlb::report_error(VLB_E_INVALID_ARG, "null argument");
    *bytes = s->total;
    return VLB_OK;
}

int vlb3_bind(vlb3_sim* s, void* ws, size_t bytes, void* stream) {
    if (!s) return vlb::report_error(VLB_E_INVALID_ARG, "null simulation");
    if (!ws || ((uintptr_t)ws & 255u) || bytes < s->total)
        return vlb::report_error(VLB_E_WORKSPACE, "workspace missing, misaligned or smaller than " +
                                                      std::to_string(s->total) + " bytes");
    s->ws = static_cast<char*>(ws);
    s->ws_bytes = bytes;
    s->stream = static_cast<hipStream_t>(stream);
    s->bound = true;
    s->inited = false;
    return VLB_OK;
}

int vlb3_set_params(vlb3_sim* s, double nu_s, double eta_p, double lambda, double kappa,
                    double Lambda_s, double Lambda_p, double Fx, double Fy, double Fz, int flags) {
    if (!s) return vlb::report_error(VLB_E_INVALID_ARG, "null simulation");
    const double v[9] = {nu_s, eta_p, lambda, kappa, Lambda_s, Lambda_p, Fx, Fy, Fz};
    for (double d : v)
        if (!std::isfinite(d)) return vlb::report_error(VLB_E_INVALID_ARG, "non-finite parameter");
    if (!(nu_s > 0) || !(kappa > 0) || !(lambda > 0) || !(eta_p >= 0) || !(Lambda_s > 0) ||
        !(Lambda_p > 0))
        return vlb::report_error(VLB_E_INVALID_ARG,
                                 "need nu_s, kappa, lambda, magic parameters > 0 and eta_p >= 0");
    if (flags & ~VLB_FLAG_NO_SOURCE) return vlb::report_error(VLB_E_INVALID_ARG, "unknown flag");
    s->nu_s = nu_s;
    s->eta_p = eta_p;
    s->lam = lambda;
    s->kappa = kappa;
    s->Ls = Lambda_s;
    s->Lp = Lambda_p;
    s->F[0] = Fx;
    s->F[1] = Fy;
    s->F[2] = Fz;
    s->flags = flags;
    s->params_set = true;
    return VLB_OK;
}

int vlb3_init_equilibrium(vlb3_sim* s, const void* const fields[10]) {
    int rc = check_ready(s);
    if (rc) return rc;
    return by_kind<InitOp>(s, fields);
}

int vlb3_step(vlb3_sim* s, int64_t n) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!s->inited) return vlb::report_error(VLB_E_STATE, "state not initialised (vlb3_init_equilibrium)");
    if (n < 0) return vlb::report_error(VLB_E_INVALID_ARG, "nsteps must be >= 0");
    return by_kind<StepOp>(s, n);
}

int vlb3_read_fields(vlb3_sim* s, void* const out[10]) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!s->inited) return vlb::report_error(VLB_E_STATE, "state not initialised (vlb3_init_equilibrium)");
    return by_kind<ReadOp>(s, out);
}

int vlb3_get_step(const vlb3_sim* s, int64_t* step) {
    if (!s || !step) return vlb::report_error(VLB_E_INVALID_ARG, "null argument");
    *step = s->step;
    return VLB_OK;
}

void vlb3_destroy(vlb3_sim* s) { delete s; }

}  // extern "C"
#endif  // VLB3_PART
