// Internal declarations shared by the host API (vlb_api.cpp) and the kernels
// (vlb_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace vlb {

enum { XM_PERIODIC = 0, XM_WALL = 1, XM_OPEN = 2 };

// Per-node geometry byte: bit 0 = the node itself is solid; bit i (1..8) = the source
// x - e_i of direction i is solid (domain wall or solid node).
enum { BIT_SELF_SOLID = 1u };

// Device descriptor of one simulation ("run").  The step kernel reads it through
// uniform (scalar) loads; a batch is an array of these.
template <class T>
struct RunDev {
    int nx, ny, pitch, xmode, ymode;
    int has_bits;       // bits plane present (walls or solid nodes)
    int has_curved;     // curved links present (bidx / bq valid)
    int uniform_force;  // 1: use Fx, Fy below; 0: force planes
    int no_source;      // constitutive source forced to zero
    int pad0;
    long long plane;    // elements per plane (ny * pitch)
    T* pop[2];          // two population buffers of 36 planes: f (9), g_xx, g_xy, g_yy (9 each)
    T* hist;            // 5 planes: S_xx, S_xy, S_yy, u_x, u_y of the previous step
    const T* force;     // 2 planes (F_x, F_y) when !uniform_force
    const uint16_t* bits;  // per node, see BIT_SELF_SOLID
    const int* bidx;    // per node: row of bq for nodes with curved links, else -1
    const T* bq;        // 8 wall fractions per boundary node (directions 1..8)
    const T* inlet;     // 4 rows of ny: u_x, A_xx, A_xy, A_yy
    // coefficients, computed in double on the host
    T c1, c2, h1, inv_ts1;  // 1 - 1/tau_s1, 1 - 1/tau_s2, 1 - 1/(2 tau_s1), 1/tau_s1
    T p1, p2, h2;           // 1 - 1/tau_p1, 1 - 1/tau_p2, 1 - 1/(2 tau_p1)
    T inv_lam, eta_over_lam;
    T Fx, Fy;
};

// Work item of the step kernel: run index, tile column, tile row.
struct Item {
    int run, tx, ty, pad;
};

struct MonitorAcc {
    double mass[4];
    double residual;  // stored as bit pattern of a non-negative double (atomic max)
    double umax;
    unsigned long long nonfinite;
    unsigned long long spd;
};

// Kernel launchers (vlb_kernels.hip).  Return hipSuccess or the launch error.
template <class T>
hipError_t launch_step(const RunDev<T>* runs_dev, const Item* items_dev, int nitems, int ty,
                       int parity, int first, hipStream_t s);
template <class T>
hipError_t launch_init(const RunDev<T>& run_host, const RunDev<T>* run_dev, const T* rho,
                       const T* ux, const T* uy, const T* axx, const T* axy, const T* ayy,
                       hipStream_t s);
template <class T>
hipError_t launch_read(const RunDev<T>& run_host, const RunDev<T>* run_dev, int parity,
                       int first, T* rho, T* ux, T* uy, T* axx, T* axy, T* ayy, hipStream_t s);
template <class T>
hipError_t launch_monitor(const RunDev<T>& run_host, const RunDev<T>* run_dev, int parity,
                          int first, T* usnap, MonitorAcc* acc, hipStream_t s);
hipError_t launch_fill_bytes(void* dst, size_t bytes, unsigned char v, hipStream_t s);
hipError_t launch_write_words(unsigned long long* dst, unsigned long long w0,
                              unsigned long long w1, unsigned long long w2,
                              unsigned long long w3, hipStream_t s);

}  // namespace vlb
