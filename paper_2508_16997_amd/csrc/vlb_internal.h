// Internal declarations shared by the host API (vlb_api.cpp) and the kernels
// (vlb_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace vlb {

// Record the thread-local error detail returned by vlb_last_error_detail; returns code.
int report_error(int code, const std::string& msg);


// XM_WET (y only): the first and last rows are wall nodes (wet-node walls).
enum { XM_PERIODIC = 0, XM_WALL = 1, XM_OPEN = 2, XM_WET = 3 };

// Per-node geometry word: bit 0 = the node itself is solid; bit i (1..8) = the source
// x - e_i of direction i is solid (domain wall or solid node).
enum { BIT_SELF_SOLID = 1u };

// Storage layout: every plane holds (ny + 2) rows of `pitch` elements.  Node (x, y) is
// element off0 + y * pitch + x with off0 = pitch + XOFF; row -1, row ny, column -1 and
// column nx around the domain are ghost slots.  XOFF = 64 keeps the rows of a 64-wide
// tile aligned to 256 bytes.
enum { XOFF = 64 };

// Kinds of fill operations (run after each step on the post-collision buffer, before
// the next step pulls from it).  One op serves direction `dir` of one fluid node.
enum {
    FILL_OUTLET = 0,   // last column, solid x0: rest equilibrium (constant)
    FILL_WALL = 1,     // half-way bounce-back: f_dir(dst) <- f_opp(src); g likewise
    FILL_CURVED = 2,   // interpolated bounce-back for f (q, far node); g as FILL_WALL
    FILL_INLET = 3     // first column, solid x0: equilibrium of the inlet profile at
                       // row `far` (constant)
};

// Constitutive closures (same values as VLB_OLDROYD_B ... VLB_FENE_P of the ABI).
enum { MODEL_OLDROYD_B = 0, MODEL_GIESEKUS = 1, MODEL_LPTT = 2, MODEL_EPTT = 3, MODEL_FENE_P = 4 };

struct FillOp {
    int dst;       // slot that the fluid node pulls direction dir from
    int src;       // fluid node x (outlet: the last-column node of that row)
    int far;       // x + e_dir for FILL_CURVED (or -1), inlet row for FILL_INLET
    int dir_kind;  // dir | kind << 8
    double q;      // wall fraction for FILL_CURVED
};

// Device descriptor of one simulation ("run").  The kernels read it through uniform
// (scalar) loads; a batch is an array of these.  S is the storage type of the
// populations and fields (float or double); all arithmetic is done in double.
template <class S>
struct RunDev {
    int nx, ny, pitch, off0, xmode, ymode;
    int has_bits;       // bits plane present (walls or solid nodes)
    int has_curved;     // curved links present (bidx / bq valid)
    int uniform_force;  // 1: use Fx, Fy below; 0: force planes
    int no_source;      // constitutive source forced to zero
    int model;          // constitutive closure (VLB_OLDROYD_B ... VLB_FENE_P)
    int wet_y;          // 1: rows 0 and ny - 1 are wet-node wall nodes (u = 0 there)
    long long plane;    // elements per plane ((ny + 2) * pitch)
    S* pop[2];          // two population buffers of 36 planes' worth: per direction i a
                        // plane of 4-vectors (f_i, g_xx,i, g_xy,i, g_yy,i), element
                        // (i * plane + slot) * 4 + lattice
    S* hist;            // 5 planes' worth: (S_xx, S_xy, S_yy, u_x) of the previous step as
                        // 4-vectors, then a plane of u_y
    S* hist_out;        // where the step writes this step's S and u (hist, except when an
                        // adjoint segment is recomputed into separate state slots)
    const S* force;     // 2 planes (F_x, F_y) when !uniform_force
    const uint16_t* bits;  // per node, see BIT_SELF_SOLID
    const int* bidx;    // per node: row of bq for nodes with curved links, else -1
    const double* bq;   // 8 wall fractions per boundary node (directions 1..8)
    const double* inlet;  // 4 rows of ny: u_x, A_xx, A_xy, A_yy
    const FillOp* fill;   // fill operations of this run
    int nfill;
    int ylw;              // 1: the curved-wall scheme YLW for f (else linear interpolation)
    int open_nebb;        // 1: wet-node NEBB open ends for f (first and last columns)
    int pad2;
    // coefficients, computed in double on the host
    double c1, c2, h1, inv_ts1;  // 1 - 1/tau_s1, 1 - 1/tau_s2, 1 - 1/(2 tau_s1), 1/tau_s1
    double p1, p2, h2;           // 1 - 1/tau_p1, 1 - 1/tau_p2, 1 - 1/(2 tau_p1)
    double inv_lam, eta_over_lam;
    double mpar;                 // closure parameter: alpha, eps or L^2 - 2 (FENE-P)
    double Fx, Fy;
};

// Work item of the step kernel: run index, tile column, tile row.
struct Item {
    int run, tx, ty, pad;
};

// Work item of the fill kernel: run index and a chunk of that run's ops.
struct FillItem {
    int run, first, count, pad;
};

// Adjoint buffers (periodic domains).  Adjoint planes use the padded layout of the
// forward state; periodic neighbours are reached by wrapping indices.
template <class S>
struct AdjDev {
    int nx, ny, pitch, off0;
    long long plane;
    S* scr;          // unused (the intermediates' two buffers are launch arguments)
    double* gF;      // 2 planes: accumulated dL/dF_x, dL/dF_y
    double* part;    // 2 per work item: accumulated dL/dlambda, dL/deta_p partials
    double* lossp;   // 1 per work item: loss partials of the seed
    const S* seed_x;  // [ny][nx] (unpadded): dL/du_x or the target u_x
    const S* seed_y;  // [ny][nx]: dL/du_y or the target u_y
    int seed_is_target;  // 1: dL/du = (u - target) / nfluid and the loss is formed
    int pad;
    double inv_nfluid;
};

struct MonitorAcc {
    double mass[4];
    double residual;  // stored as bit pattern of a non-negative double (atomic max)
    double umax;
    unsigned long long nonfinite;
    unsigned long long spd;
};

// Kernel launchers (vlb_kernels.hip).  Return hipSuccess or the launch error.
// streaming != 0 selects non-temporal stores of the post-collision state; waves (3 or 4)
// the register budget of the single-precision step kernel.
template <class S>
hipError_t launch_step(const RunDev<S>* runs_dev, const Item* items_dev, int nitems, int ty,
                       int parity, int first, int streaming, int waves, hipStream_t s);
// Persistent batch form (vlb_batch.hip): one cooperative launch runs nsteps steps (step,
// grid barrier, fills, grid barrier) over the same work and fill lists.  queues: device
// array of 2 * kBatchQueues ints, zero before the first launch and left zero by each.
constexpr int kBatchQueues = 8;
template <class S>
hipError_t launch_batch(const RunDev<S>* runs_dev, const Item* items_dev, int nitems,
                        const FillItem* fitems_dev, int nfitems, int nsteps, int ty, int parity,
                        int first, int streaming, int* queues, hipStream_t s);
template <class S>
hipError_t launch_fill(const RunDev<S>* runs_dev, const FillItem* items_dev, int nitems,
                       int parity, hipStream_t s);
template <class S>
hipError_t launch_init(const RunDev<S>& run_host, const RunDev<S>* run_dev, const S* rho,
                       const S* ux, const S* uy, const S* axx, const S* axy, const S* ayy,
                       hipStream_t s);
template <class S>
hipError_t launch_read(const RunDev<S>& run_host, const RunDev<S>* run_dev, int parity,
                       int first, S* rho, S* ux, S* uy, S* axx, S* axy, S* ayy, hipStream_t s);
template <class S>
hipError_t launch_read_history(const RunDev<S>& run_host, const RunDev<S>* run_dev, S* sxx, S* sxy,
                               S* syy, S* uxp, S* uyp, hipStream_t s);
// Deterministic two-pass reduction; part holds 8 doubles per 64 x 4 block of nodes.
template <class S>
hipError_t launch_monitor(const RunDev<S>& run_host, const RunDev<S>* run_dev, int parity,
                          int first, S* usnap, double* part, MonitorAcc* acc, hipStream_t s);
template <class S>
hipError_t launch_adj_seed(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                           int nitems, int ty, const S* src, int pull, S* aout, hipStream_t s);
// One reverse step: walls: the run has geometry bits (walls, solids), 0 selects the
// periodic kernels; fused: the hydrodynamic adjoints of ain are formed in the launch from
// the later step's intermediates scr_in (every reverse step but the first); the step's
// own intermediates go to scr_out.
template <class S>
hipError_t launch_adj_step(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                           int nitems, int ty, int first, int walls, int fused, const S* ain,
                           S* aout, const S* scr_in, S* scr_out, hipStream_t s);
// The gather of the last reverse step (step 0): its hydrodynamic adjoints into aout and
// its dL/dF, from its intermediates scr.
template <class S>
hipError_t launch_adj_gather(const RunDev<S>* run_dev, const AdjDev<S>* adj_dev, const Item* items,
                             int nitems, int ty, int walls, const S* scr, S* aout, hipStream_t s);
// Momentum-exchange force: per block of 256 boundary links, 2 partial sums (F_x, F_y).
template <class S>
hipError_t launch_drag(const RunDev<S>* run_dev, const int* links, int nlinks, int circle,
                       int parity, double* part, hipStream_t s);
hipError_t launch_fill_bytes(void* dst, size_t bytes, unsigned char v, hipStream_t s);
hipError_t launch_write_words(unsigned long long* dst, unsigned long long w0,
                              unsigned long long w1, unsigned long long w2,
                              unsigned long long w3, hipStream_t s);

}  // namespace vlb
