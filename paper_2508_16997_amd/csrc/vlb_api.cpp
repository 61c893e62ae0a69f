// vlb_api.cpp -- host side of the C ABI declared in include/vlb.h.
//
// Geometry (node classes, wall links, wall fractions) is built here on the host; the
// rules must match any other implementation bit for bit, so the wall fraction uses the
// fixed expression order below and this file is compiled without FP contraction.
// All device memory comes from the caller's workspace; the library only carves it.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "vlb.h"
#include "vlb_internal.h"

namespace {

// roctx range around an entry point that enqueues device work: shows up as a named
// region in rocprofv3 --marker-trace timelines, costs one call when no tool listens.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

thread_local std::string g_detail;

int fail(int code, const std::string& msg) {
    g_detail = msg;
    return code;
}

#define VLB_HIP(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(VLB_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// D2Q9 in the paper's order (Sec. 3.1).
const int EXH[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int EYH[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const int OPPH[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Link {
    int32_t node;
    int8_t dir;
    double q;
};

template <class T>
using Run = vlb::RunDev<T>;

}  // namespace

int vlb::report_error(int code, const std::string& msg) { return fail(code, msg); }

static_assert(vlb::MODEL_GIESEKUS == VLB_GIESEKUS && vlb::MODEL_LPTT == VLB_LPTT &&
                  vlb::MODEL_EPTT == VLB_EPTT && vlb::MODEL_FENE_P == VLB_FENE_P,
              "closure codes of the ABI and the kernels differ");

struct vlb_sim {
    int nx = 0, ny = 0, xmode = 0, ymode = 0, prec = 0, pitch = 0, off0 = 0;
    long long plane = 0;
    size_t esz = 4;
    std::vector<uint8_t> solid;     // [ny][nx]
    std::vector<int> circle_of;     // [ny][nx]
    std::vector<double> circles;    // xc, yc, R
    std::vector<uint16_t> bits;     // padded plane
    std::vector<Link> links;
    std::vector<int> drag_links;    // per link: slot of the fluid node, direction, circle or -1
    std::vector<int> bidx;          // padded plane, curved only
    std::vector<vlb::FillOp> fill;  // boundary links served by the fill kernel
    std::vector<vlb::FillItem> fill_items;
    std::vector<double> bq;         // 8 per boundary node
    int nbq = 0;
    bool has_bits = false, has_curved = false;

    // binding
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    size_t off_pop[2] = {0, 0}, off_hist = 0, off_force = 0, off_usnap = 0, off_inlet = 0,
           off_bq = 0, off_bits = 0, off_bidx = 0, off_run = 0, off_items = 0, off_mon = 0, off_monpart = 0, off_drag = 0, off_dragpart = 0,
           off_fill = 0, off_fill_items = 0, total = 0;

    std::vector<vlb::Item> items;
    int nitems = 0;
    int ty = 4;
    int items_cap = 0;

    vlb_params params{};
    bool params_set = false, force_field = false, inited = false;
    std::vector<double> inlet;  // 4 * ny
    int parity = 0, first = 1;
    int64_t step = 0;

    uint64_t version = 0;  // bumped whenever the device descriptor is rewritten

    // record of the last vlb_adjoint_forward (checkpoints live in the caller's workspace)
    struct {
        bool valid = false;
        char* ws = nullptr;
        size_t bytes = 0;
        int64_t nsteps = 0, step0 = 0;
        int stride = 0, first0 = 0, ty = 0;
        uint64_t version = 0;
    } adj;
    int graph_chunk = 0;
    int store_mode = 0;  // 0 auto (by working-set size), 1 cached stores, 2 streaming stores
    int sched_order = 0;  // tile order: 0 auto, 1 XCD bands, 2 row-major
    int sched_waves = 0;  // register budget of the FP32 step kernel: 0 auto, 3 or 4 waves
    hipGraphExec_t graph[2] = {nullptr, nullptr};

    template <class T>
    T* dptr(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

// A batch: many bound simulations of one precision advanced by one step launch and one
// fill launch per time step over the concatenated work lists.
struct vlb_batch {
    std::vector<vlb_sim*> sims;
    int prec = 0, ty = 4, streaming = 0;
    int sched_order = 0, sched_waves = 0;  // as for a simulation
    bool resident = true;                  // the members' state fits the last-level cache
    std::vector<vlb::Item> tiles;          // the members' tiles, member by member
    char* ws = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    size_t off_runs = 0, off_items = 0, off_fill_items = 0, off_queues = 0, total = 0;
    std::vector<vlb::Item> items;
    std::vector<vlb::FillItem> fill_items;
    int graph_chunk = 0;
    int persistent = 0;  // 1: cooperative persistent launches (launch_batch)
    int64_t step = 0;  // step count of every member, as advanced by the batch
    std::vector<uint64_t> versions;  // member descriptor versions last copied
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int scratch_dev = -1;  // >= 0: lists live in that device's static scratch (noalloc form)
};

namespace {

int wrap(int v, int n) { return ((v % n) + n) % n; }

// Wall fraction of the link from fluid node (x, y) in direction d toward the circle c:
// smallest root of |x + t e_d - c|^2 = R^2.
double circle_q(const vlb_sim* s, int x, int y, int d, int c) {
    const double dx = (double)EXH[d], dy = (double)EYH[d];
    const double px = (double)x - s->circles[3 * c], py = (double)y - s->circles[3 * c + 1];
    const double r = s->circles[3 * c + 2];
    const double a = dx * dx + dy * dy;
    const double b = 2.0 * (px * dx + py * dy);
    const double cc = px * px + py * py - r * r;
    const double disc = b * b - 4.0 * a * cc;
    return (-b - std::sqrt(disc)) / (2.0 * a);
}

// Node classes, geometry bits, links, and the curved-link table.
void build_geometry(vlb_sim* s, const uint8_t* mask) {
    const int nx = s->nx, ny = s->ny;
    const int nc = (int)s->circles.size() / 3;
    s->solid.assign((size_t)nx * ny, 0);
    s->circle_of.assign((size_t)nx * ny, -1);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t n = (size_t)y * nx + x;
            if (mask && mask[n]) s->solid[n] = 1;
            for (int c = 0; c < nc; ++c) {
                const double dx = (double)x - s->circles[3 * c];
                const double dy = (double)y - s->circles[3 * c + 1];
                const double r = s->circles[3 * c + 2];
                if (dx * dx + dy * dy <= r * r) {
                    s->solid[n] = 1;
                    if (s->circle_of[n] < 0) s->circle_of[n] = c;
                }
            }
        }
    s->bits.assign((size_t)s->plane, 0);
    s->links.clear();
    s->drag_links.clear();
    bool any_bits = false, curved = false;
    std::vector<double> qnode(9);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t n = (size_t)y * nx + x;
            const size_t pp = (size_t)s->off0 + (size_t)y * s->pitch + x;
            if (s->solid[n]) {
                s->bits[pp] = vlb::BIT_SELF_SOLID;
                any_bits = true;
                continue;
            }
            uint16_t b = 0;
            for (int d = 1; d < 9; ++d) {
                // neighbour x + e_d (the source of direction opp(d))
                int xn = x + EXH[d], yn = y + EYH[d];
                const bool xout = xn < 0 || xn >= nx, yout = yn < 0 || yn >= ny;
                bool is_solid = false;
                double q = 0.5;
                int cid = -1;
                if ((yout && (s->ymode == VLB_WALL || s->ymode == VLB_WET)) ||
                    (xout && s->xmode == VLB_WALL)) {
                    is_solid = true;
                } else {
                    if (yout) yn = wrap(yn, ny);
                    bool ghost = false;
                    if (xout) {
                        if (s->xmode == VLB_PERIODIC) xn = wrap(xn, nx);
                        else ghost = true;  // inlet / outlet ghost column
                    }
                    if (!ghost) {
                        const size_t m = (size_t)yn * nx + xn;
                        if (s->solid[m]) {
                            is_solid = true;
                            if (s->circle_of[m] >= 0) {
                                q = circle_q(s, x, y, d, s->circle_of[m]);
                                curved = true;
                                cid = s->circle_of[m];
                            }
                        }
                    }
                }
                if (is_solid) {
                    b |= (uint16_t)(1u << OPPH[d]);
                    s->links.push_back(Link{(int32_t)n, (int8_t)d, q});
                    s->drag_links.insert(s->drag_links.end(), {(int)pp, d, cid});
                }
            }
            s->bits[pp] = b;
            if (b) any_bits = true;
        }
    s->has_bits = any_bits;
    s->has_curved = curved;
    s->bidx.clear();
    s->bq.clear();
    s->nbq = 0;
    if (curved) {
        s->bidx.assign((size_t)s->plane, -1);
        // links are in (node, dir) order; group them per node
        size_t i = 0;
        while (i < s->links.size()) {
            const int32_t n = s->links[i].node;
            const int x = n % nx, y = n / nx;
            std::fill(qnode.begin(), qnode.end(), 0.5);
            for (; i < s->links.size() && s->links[i].node == n; ++i)
                qnode[OPPH[s->links[i].dir]] = s->links[i].q;  // indexed by unknown direction
            s->bidx[(size_t)s->off0 + (size_t)y * s->pitch + x] = s->nbq++;
            for (int k = 1; k < 9; ++k) s->bq.push_back(qnode[k]);
        }
    }
}

// One fill op per fluid node and direction whose source x - e_i is not a fluid node
// of the domain: the op writes into the slot of x - e_i (ghost or solid node) the value
// the boundary rule gives for that link.
void build_fill(vlb_sim* s) {
    const int nx = s->nx, ny = s->ny;
    s->fill.clear();
    auto slot = [&](int xx, int yy) { return s->off0 + yy * s->pitch + xx; };
    auto fluid_at = [&](int xx, int yy, int* idx) -> bool {
        // in-domain fluid node after periodic wrap
        if (yy < 0 || yy >= ny) {
            if (s->ymode != VLB_PERIODIC) return false;
            yy = wrap(yy, ny);
        }
        if (xx < 0 || xx >= nx) {
            if (s->xmode != VLB_PERIODIC) return false;
            xx = wrap(xx, nx);
        }
        if (s->solid[(size_t)yy * nx + xx]) return false;
        *idx = slot(xx, yy);
        return true;
    };
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (s->solid[(size_t)y * nx + x]) continue;
            const int p = slot(x, y);
            const uint16_t b = s->bits[(size_t)p];
            int bi = -1;
            if (s->has_curved) bi = s->bidx[(size_t)p];
            for (int i = 1; i < 9; ++i) {
                const int xs = x - EXH[i], ys = y - EYH[i];
                vlb::FillOp op{slot(xs, ys), p, -1, i, 0.5};
                if (b & (1u << i)) {
                    const double q = bi >= 0 ? s->bq[(size_t)bi * 8 + (i - 1)] : 0.5;
                    int far = -1;
                    const bool has_far = q != 0.5 && fluid_at(x + EXH[i], y + EYH[i], &far);
                    if (q == 0.5 || (q < 0.5 && !has_far)) {
                        op.dir_kind = i | (vlb::FILL_WALL << 8);
                    } else {
                        op.dir_kind = i | (vlb::FILL_CURVED << 8);
                        op.q = q;
                        op.far = has_far ? far : -1;
                    }
                    s->fill.push_back(op);
                    continue;
                }
                const bool xout = xs < 0 || xs >= nx, yout = ys < 0 || ys >= ny;
                if (!xout && !yout) continue;  // ordinary pull from a fluid node
                const int yw = yout ? wrap(ys, ny) : ys;
                if (xout && s->xmode == VLB_OPEN) {
                    // the extrapolation node x0 (same row as the ghost, first or last
                    // column) writes this ghost itself in the step kernel; only ghosts of
                    // a solid x0 (constant equilibrium values) stay in the fill list
                    const int x0c = xs < 0 ? 0 : nx - 1;
                    if (!s->solid[(size_t)yw * nx + x0c]) continue;
                    if (xs < 0) {
                        op.dir_kind = i | (vlb::FILL_INLET << 8);
                        op.far = yw;
                        op.src = p;
                    } else {
                        op.dir_kind = i | (vlb::FILL_OUTLET << 8);
                        op.src = slot(nx - 1, yw);
                    }
                } else {
                    // periodic image: written by the step kernel's edge stores
                    continue;
                }
                s->fill.push_back(op);
            }
        }
    // Group the ops by kind (node order kept within a kind) so that a wavefront runs
    // one boundary rule instead of serialising several.
    std::stable_sort(s->fill.begin(), s->fill.end(), [](const vlb::FillOp& a, const vlb::FillOp& b) {
        return (a.dir_kind >> 8) < (b.dir_kind >> 8);
    });
    s->fill_items.clear();
    for (int f = 0; f < (int)s->fill.size(); f += 256)
        s->fill_items.push_back(vlb::FillItem{0, f, std::min(256, (int)s->fill.size() - f), 0});
}

// Work items in an XCD-aware order: consecutive workgroups go round-robin to the 8
// XCDs, so block b is given tile (start of XCD b % 8) + b / 8 and every XCD sweeps a
// contiguous band of tiles (shared halo rows stay in one L2).
// Launch order of a tile list (tiles of each run row-major, runs one after another).
// Consecutive workgroups go round-robin to the 8 XCDs, so with a list split into 8
// bands, block b taking entry (start of band b % 8) + b / 8 makes XCD b % 8 sweep band
// b % 8, in list order.
//   XCD bands (order 1): the bands are contiguous runs of the row-major list, so each XCD
//     sweeps a band of tile rows and the halo rows it pulls meet in its own L2 -- the
//     better order while the state is cache resident.
//   Row-major (order 2): the list itself, the whole chip sweeping the grid together so
//     that all XCDs stream from the same rows of memory.
//   Column strips (order 3): each run's tile columns cut into 8 strips, the list strip by
//     strip (row-major inside a strip), then XCD bands: every XCD owns a strip, its
//     neighbours in x and y share its L2, and all XCDs move down the rows together.
void order_tiles(const std::vector<vlb::Item>& tiles, int order, std::vector<vlb::Item>& out) {
    const int n = (int)tiles.size(), nxcd = 8;
    out.resize(n);
    if (order == 2) {
        out = tiles;
        return;
    }
    std::vector<vlb::Item> list = tiles;
    if (order == 3) {
        // strip of a tile: its column's eighth of the run's tile columns
        int ntx_max = 0;
        std::vector<int> ntx;  // tile columns of each run
        for (const vlb::Item& t : tiles) {
            if (t.run >= (int)ntx.size()) ntx.resize(t.run + 1, 0);
            ntx[t.run] = std::max(ntx[t.run], t.tx + 1);
            ntx_max = std::max(ntx_max, t.tx + 1);
        }
        (void)ntx_max;
        auto strip = [&](const vlb::Item& t) { return (t.tx * nxcd) / ntx[t.run]; };
        std::stable_sort(list.begin(), list.end(), [&](const vlb::Item& a, const vlb::Item& b) {
            if (a.run != b.run) return a.run < b.run;
            const int sa = strip(a), sb = strip(b);
            if (sa != sb) return sa < sb;
            if (a.ty != b.ty) return a.ty < b.ty;
            return a.tx < b.tx;
        });
    }
    std::vector<int> start(nxcd + 1, 0);
    for (int k = 0; k < nxcd; ++k) start[k + 1] = start[k] + n / nxcd + (k < n % nxcd ? 1 : 0);
    for (int b = 0; b < n; ++b) out[b] = list[start[b % nxcd] + b / nxcd];
}

// The state of both population buffers fits the 256 MB last-level cache.
bool resident_state(const vlb_sim* s) {
    return 2.0 * 36.0 * (double)s->nx * (double)s->ny * (double)s->esz <= 192.0 * 1024 * 1024;
}
// Schedule in effect: explicit choices, else XCD bands for a cache-resident state and
// row-major tiles once it streams from HBM (measured on the 512^2 and 4096 x 1024 grids:
// bands 17.5 us against 18.2 us row-major; row-major 268 us against 275 us in strips and
// 277 us in bands), four waves per SIMD.
int effective_order(int order, bool resident) { return order ? order : (resident ? 1 : 2); }
int step_waves(int waves, bool resident) { (void)resident; return waves ? waves : 4; }

void build_items(vlb_sim* s) {
    const int ntx = (s->nx + 63) / 64, nty = (s->ny + s->ty - 1) / s->ty;
    const int n = ntx * nty;
    std::vector<vlb::Item> tiles(n);
    for (int t = 0; t < n; ++t) tiles[t] = vlb::Item{0, t % ntx, t / ntx, 0};
    order_tiles(tiles, effective_order(s->sched_order, resident_state(s)), s->items);
    s->nitems = n;
}

void layout(vlb_sim* s) {
    const size_t e = s->esz;
    const size_t plane_b = (size_t)s->plane * e;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + bytes); return r; };
    s->off_pop[0] = take(36 * plane_b);
    s->off_pop[1] = take(36 * plane_b);
    s->off_hist = take(5 * plane_b);
    s->off_force = take(2 * plane_b);
    s->off_usnap = take(2 * (size_t)s->nx * s->ny * e);
    s->off_inlet = take(4 * (size_t)s->ny * sizeof(double));
    s->off_bq = take(std::max<size_t>(1, (size_t)s->nbq * 8) * sizeof(double));
    s->off_bits = take((size_t)s->plane * sizeof(uint16_t));
    s->off_bidx = take(s->has_curved ? (size_t)s->plane * sizeof(int) : 256);
    s->off_run = take(sizeof(Run<double>));
    s->items_cap = ((s->nx + 63) / 64) * s->ny;  // enough for any tile height >= 1
    s->off_items = take((size_t)s->items_cap * sizeof(vlb::Item));
    s->off_mon = take(sizeof(vlb::MonitorAcc));
    s->off_monpart = take(8 * sizeof(double) * (size_t)((s->nx + 63) / 64) * (size_t)((s->ny + 3) / 4));
    s->off_drag = take(std::max<size_t>(3, s->drag_links.size()) * sizeof(int));
    s->off_dragpart = take(2 * sizeof(double) * std::max<size_t>(1, (s->links.size() + 255) / 256));
    s->off_fill = take(std::max<size_t>(1, s->fill.size()) * sizeof(vlb::FillOp));
    s->off_fill_items = take(std::max<size_t>(1, s->fill_items.size()) * sizeof(vlb::FillItem));
    s->total = o;
}

template <class T>
Run<T> make_run(const vlb_sim* s) {
    Run<T> r{};
    r.nx = s->nx; r.ny = s->ny; r.pitch = s->pitch; r.off0 = s->off0;
    r.xmode = s->xmode; r.ymode = s->ymode;
    r.wet_y = s->ymode == VLB_WET ? 1 : 0;
    r.has_bits = s->has_bits ? 1 : 0;
    r.has_curved = s->has_curved ? 1 : 0;
    r.uniform_force = s->force_field ? 0 : 1;
    r.no_source = (s->params.flags & VLB_FLAG_NO_SOURCE) ? 1 : 0;
    r.ylw = (s->params.flags & VLB_FLAG_CURVED_YLW) ? 1 : 0;
    r.open_nebb = (s->params.flags & VLB_FLAG_OPEN_NEBB) ? 1 : 0;
    r.plane = s->plane;
    r.pop[0] = s->dptr<T>(s->off_pop[0]);
    r.pop[1] = s->dptr<T>(s->off_pop[1]);
    r.hist = s->dptr<T>(s->off_hist);
    r.hist_out = r.hist;
    r.force = s->dptr<T>(s->off_force);
    r.bits = s->dptr<uint16_t>(s->off_bits);
    r.bidx = s->has_curved ? s->dptr<int>(s->off_bidx) : nullptr;
    r.bq = s->dptr<double>(s->off_bq);
    r.inlet = s->dptr<double>(s->off_inlet);
    r.fill = s->dptr<vlb::FillOp>(s->off_fill);
    r.nfill = (int)s->fill.size();
    const vlb_params& p = s->params;
    // relaxation times from the transport relations (Sec. 3.1-3.2), c_s^2 = 1/3
    const double ts1 = 3.0 * p.nu_s + 0.5;
    const double ts2 = p.Lambda_s / (3.0 * p.nu_s) + 0.5;
    const double tp1 = 3.0 * p.kappa + 0.5;
    const double tp2 = p.Lambda_p / (3.0 * p.kappa) + 0.5;
    r.c1 = (ts1 - 1.0) / ts1;
    r.c2 = (ts2 - 1.0) / ts2;
    r.h1 = (3.0 * p.nu_s) / ts1;  // 1 - 1/(2 tau_s1) without cancellation
    r.inv_ts1 = 1.0 / ts1;
    r.p1 = (tp1 - 1.0) / tp1;
    r.p2 = (tp2 - 1.0) / tp2;
    r.h2 = (3.0 * p.kappa) / tp1;
    r.inv_lam = 1.0 / p.lambda;
    r.eta_over_lam = p.eta_p / p.lambda;
    r.model = p.model;
    r.mpar = p.model == VLB_FENE_P ? p.model_param - 2.0 : (p.model == VLB_OLDROYD_B ? 0.0 : p.model_param);
    r.Fx = p.Fx;
    r.Fy = p.Fy;
    return r;
}

template <class T>
__global__ void k_store_run(Run<T> v, Run<T>* dst) {
    if (threadIdx.x == 0) *dst = v;
}

int upload_run(vlb_sim* s) {
    ++s->version;
    if (s->prec == VLB_FP32) {
        hipLaunchKernelGGL((k_store_run<float>), dim3(1), dim3(64), 0, s->stream, make_run<float>(s),
                           s->dptr<Run<float>>(s->off_run));
    } else {
        hipLaunchKernelGGL((k_store_run<double>), dim3(1), dim3(64), 0, s->stream,
                           make_run<double>(s), s->dptr<Run<double>>(s->off_run));
    }
    VLB_HIP(hipGetLastError());
    return VLB_OK;
}

int upload_items(vlb_sim* s) {
    build_items(s);
    VLB_HIP(hipMemcpyAsync(s->ws + s->off_items, s->items.data(),
                           s->items.size() * sizeof(vlb::Item), hipMemcpyHostToDevice, s->stream));
    VLB_HIP(hipStreamSynchronize(s->stream));
    return VLB_OK;
}

void drop_graphs(vlb_sim* s) {
    for (auto& g : s->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

int check_bound(const vlb_sim* s) {
    if (!s) return fail(VLB_E_INVALID_ARG, "null simulation");
    if (!s->bound) return fail(VLB_E_STATE, "workspace not bound (vlb_bind)");
    return VLB_OK;
}

int check_ready(const vlb_sim* s) {
    int rc = check_bound(s);
    if (rc) return rc;
    if (!s->params_set) return fail(VLB_E_STATE, "parameters not set (vlb_set_params)");
    if (!s->inited) return fail(VLB_E_STATE, "state not initialised (vlb_init_equilibrium)");
    return VLB_OK;
}

// Non-temporal stores pay off once both population buffers exceed the last-level
// cache (256 MB Infinity Cache); below that the state stays cache resident.
int streaming(const vlb_sim* s) {
    if (s->store_mode == 1) return 0;
    if (s->store_mode == 2) return 1;
    const double bytes = 2.0 * 36.0 * (double)s->nx * (double)s->ny * (double)s->esz;
    return bytes > 192.0 * 1024 * 1024 ? 1 : 0;
}

template <class T>
int launch_steps(vlb_sim* s, int64_t n) {
    const Run<T>* rd = s->dptr<Run<T>>(s->off_run);
    const vlb::Item* it = s->dptr<vlb::Item>(s->off_items);
    const vlb::FillItem* fi = s->dptr<vlb::FillItem>(s->off_fill_items);
    for (int64_t k = 0; k < n; ++k) {
        VLB_HIP(vlb::launch_step<T>(rd, it, s->nitems, s->ty, s->parity, s->first, streaming(s),
                                    step_waves(s->sched_waves, resident_state(s)), s->stream));
        s->parity ^= 1;
        s->first = 0;
        ++s->step;
        VLB_HIP(vlb::launch_fill<T>(rd, fi, (int)s->fill_items.size(), s->parity, s->stream));
    }
    return VLB_OK;
}

// hipGraph of 2*chunk steps starting from buffer `par` (parity returns to par).
template <class T>
int graph_for(vlb_sim* s, int par, hipGraphExec_t* out) {
    if (s->graph[par]) { *out = s->graph[par]; return VLB_OK; }
    hipGraph_t g = nullptr;
    VLB_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    const Run<T>* rd = s->dptr<Run<T>>(s->off_run);
    const vlb::Item* it = s->dptr<vlb::Item>(s->off_items);
    hipError_t err = hipSuccess;
    const vlb::FillItem* fi = s->dptr<vlb::FillItem>(s->off_fill_items);
    int p = par;
    for (int k = 0; k < 2 * s->graph_chunk && err == hipSuccess; ++k) {
        err = vlb::launch_step<T>(rd, it, s->nitems, s->ty, p, 0, streaming(s),
                                  step_waves(s->sched_waves, resident_state(s)), s->stream);
        p ^= 1;
        if (err == hipSuccess) err = vlb::launch_fill<T>(rd, fi, (int)s->fill_items.size(), p, s->stream);
    }
    hipError_t e2 = hipStreamEndCapture(s->stream, &g);
    if (err != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(VLB_E_HIP, std::string("graph capture: ") +
                                   hipGetErrorString(err != hipSuccess ? err : e2));
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return fail(VLB_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e3));
    s->graph[par] = ex;
    *out = ex;
    return VLB_OK;
}

template <class T>
int do_step(vlb_sim* s, int64_t n) {
    if (s->first && n > 0) {
        int rc = launch_steps<T>(s, 1);
        if (rc) return rc;
        --n;
    }
    if (s->graph_chunk > 0 && s->stream != nullptr) {
        const int64_t per = 2 * (int64_t)s->graph_chunk;
        while (n >= per) {
            hipGraphExec_t ex = nullptr;
            int rc = graph_for<T>(s, s->parity, &ex);
            if (rc) return rc;
            VLB_HIP(hipGraphLaunch(ex, s->stream));
            s->step += per;
            n -= per;
        }
    }
    return launch_steps<T>(s, n);
}

}  // namespace

extern "C" {

const char* vlb_error_string(int status) {
    switch (status) {
        case VLB_OK: return "ok";
        case VLB_E_INVALID_ARG: return "invalid argument";
        case VLB_E_WORKSPACE: return "workspace missing or too small";
        case VLB_E_HIP: return "HIP runtime error";
        case VLB_E_NONFINITE: return "non-finite value (numerical breakdown)";
        case VLB_E_STATE: return "call out of order";
        case VLB_E_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* vlb_last_error_detail(void) { return g_detail.c_str(); }

int vlb_create(const vlb_grid* g, vlb_sim** out) {
    if (!g || !out) return fail(VLB_E_INVALID_ARG, "null argument");
    *out = nullptr;
    if (g->nx < 1 || g->ny < 1 || ((long long)g->nx + 129) * (g->ny + 2) >= (1LL << 31) / 64)
        return fail(VLB_E_INVALID_ARG, "grid size out of range");
    if (g->xmode < VLB_PERIODIC || g->xmode > VLB_OPEN || g->ymode < VLB_PERIODIC ||
        g->ymode > VLB_WET || g->ymode == VLB_OPEN)
        return fail(VLB_E_INVALID_ARG,
                    "boundary mode out of range (ymode cannot be open, xmode cannot be wet)");
    if (g->ymode == VLB_WET && g->ny < 5)
        return fail(VLB_E_INVALID_ARG, "wet-node walls need ny >= 5");
    if ((g->xmode == VLB_OPEN || g->xmode == VLB_PERIODIC) && g->nx < 2)
        return fail(VLB_E_INVALID_ARG, "periodic or open x needs nx >= 2");
    if (g->ymode == VLB_PERIODIC && g->ny < 2)
        return fail(VLB_E_INVALID_ARG, "periodic y needs ny >= 2");
    if (g->precision != VLB_FP32 && g->precision != VLB_FP64)
        return fail(VLB_E_INVALID_ARG, "precision must be VLB_FP32 or VLB_FP64");
    if (g->ncircles < 0 || (g->ncircles > 0 && !g->circles))
        return fail(VLB_E_INVALID_ARG, "circles");
    for (int c = 0; c < g->ncircles; ++c)
        if (!(g->circles[3 * c + 2] > 0) || !std::isfinite(g->circles[3 * c]) ||
            !std::isfinite(g->circles[3 * c + 1]))
            return fail(VLB_E_INVALID_ARG, "circle radius must be > 0 and centre finite");
    vlb_sim* s = new (std::nothrow) vlb_sim();
    if (!s) return fail(VLB_E_INVALID_ARG, "out of host memory");
    s->nx = g->nx;
    s->ny = g->ny;
    s->xmode = g->xmode;
    s->ymode = g->ymode;
    s->prec = g->precision;
    s->esz = g->precision == VLB_FP32 ? 4 : 8;
    s->pitch = ((g->nx + vlb::XOFF + 1 + 63) / 64) * 64;
    s->off0 = s->pitch + vlb::XOFF;
    s->plane = (long long)s->pitch * (g->ny + 2);
    if (g->ncircles) s->circles.assign(g->circles, g->circles + 3 * g->ncircles);
    build_geometry(s, g->solid_mask);
    if (s->ymode == VLB_WET) {
        // the wall rows and the two rows next to each (one-sided differences at the
        // wall nodes) must be fluid
        for (int y : {0, 1, 2, s->ny - 3, s->ny - 2, s->ny - 1})
            for (int x = 0; x < s->nx; ++x)
                if (s->solid[(size_t)y * s->nx + x]) {
                    delete s;
                    return fail(VLB_E_INVALID_ARG,
                                "wet-node walls: rows 0-2 and ny-3..ny-1 must be fluid");
                }
    }
    build_fill(s);
    s->inlet.assign(4 * (size_t)g->ny, 0.0);
    for (int y = 0; y < g->ny; ++y) { s->inlet[g->ny + y] = 1.0; s->inlet[3 * g->ny + y] = 1.0; }
    layout(s);
    *out = s;
    return VLB_OK;
}

void vlb_destroy(vlb_sim* s) {
    if (!s) return;
    drop_graphs(s);
    delete s;
}

int vlb_workspace_bytes(const vlb_sim* s, size_t* bytes) {
    if (!s || !bytes) return fail(VLB_E_INVALID_ARG, "null argument");
    *bytes = s->total;
    return VLB_OK;
}

int vlb_geometry(const vlb_sim* s, uint8_t* cls, int32_t* lnode, int8_t* ldir, double* lq,
                 int cap, int* nlinks) {
    if (!s) return fail(VLB_E_INVALID_ARG, "null simulation");
    if (cap < 0 || (cap > 0 && (!lnode || !ldir || !lq)))
        return fail(VLB_E_INVALID_ARG, "link arrays");
    if (cls) {
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                const size_t n = (size_t)y * s->nx + x;
                const uint16_t b = s->bits[(size_t)s->off0 + (size_t)y * s->pitch + x];
                cls[n] = s->solid[n] ? VLB_NODE_SOLID
                                     : ((b & 0x1FE) ? VLB_NODE_BOUNDARY : VLB_NODE_FLUID);
            }
    }
    const int cnt = (int)s->links.size();
    for (int i = 0; i < cnt && i < cap; ++i) {
        lnode[i] = s->links[i].node;
        ldir[i] = s->links[i].dir;
        lq[i] = s->links[i].q;
    }
    if (nlinks) *nlinks = cnt;
    return VLB_OK;
}

int vlb_bind(vlb_sim* s, void* ws, size_t bytes, void* stream) {
    if (!s) return fail(VLB_E_INVALID_ARG, "null simulation");
    if (!ws) return fail(VLB_E_WORKSPACE, "null workspace");
    if (((uintptr_t)ws & 255u) != 0) return fail(VLB_E_WORKSPACE, "workspace not 256-byte aligned");
    if (bytes < s->total)
        return fail(VLB_E_WORKSPACE, "workspace too small: need " + std::to_string(s->total) +
                                         " bytes, got " + std::to_string(bytes));
    drop_graphs(s);
    s->ws = static_cast<char*>(ws);
    s->ws_bytes = bytes;
    s->stream = static_cast<hipStream_t>(stream);
    s->bound = true;
    s->inited = false;
    VLB_HIP(vlb::launch_fill_bytes(s->ws, s->total, 0, s->stream));
    if (!s->fill.empty()) {
        VLB_HIP(hipMemcpyAsync(s->ws + s->off_fill, s->fill.data(), s->fill.size() * sizeof(vlb::FillOp),
                               hipMemcpyHostToDevice, s->stream));
        VLB_HIP(hipMemcpyAsync(s->ws + s->off_fill_items, s->fill_items.data(),
                               s->fill_items.size() * sizeof(vlb::FillItem), hipMemcpyHostToDevice,
                               s->stream));
    }
    VLB_HIP(hipMemcpyAsync(s->ws + s->off_bits, s->bits.data(), s->bits.size() * sizeof(uint16_t),
                           hipMemcpyHostToDevice, s->stream));
    if (!s->drag_links.empty())
        VLB_HIP(hipMemcpyAsync(s->ws + s->off_drag, s->drag_links.data(),
                               s->drag_links.size() * sizeof(int), hipMemcpyHostToDevice, s->stream));
    if (s->has_curved) {
        VLB_HIP(hipMemcpyAsync(s->ws + s->off_bidx, s->bidx.data(), s->bidx.size() * sizeof(int),
                               hipMemcpyHostToDevice, s->stream));
    }
    // wall fractions and inlet rows (double)
    if (!s->bq.empty())
        VLB_HIP(hipMemcpyAsync(s->ws + s->off_bq, s->bq.data(), s->bq.size() * sizeof(double),
                               hipMemcpyHostToDevice, s->stream));
    VLB_HIP(hipMemcpyAsync(s->ws + s->off_inlet, s->inlet.data(), s->inlet.size() * sizeof(double),
                           hipMemcpyHostToDevice, s->stream));
    VLB_HIP(hipStreamSynchronize(s->stream));
    int rc = VLB_OK;
    rc = upload_items(s);
    if (rc) return rc;
    if (s->params_set) return upload_run(s);
    return VLB_OK;
}

int vlb_set_params(vlb_sim* s, const vlb_params* p) {
    if (!s || !p) return fail(VLB_E_INVALID_ARG, "null argument");
    const double v[8] = {p->nu_s, p->eta_p, p->lambda, p->kappa, p->Lambda_s, p->Lambda_p, p->Fx, p->Fy};
    for (double d : v)
        if (!std::isfinite(d)) return fail(VLB_E_INVALID_ARG, "non-finite parameter");
    if (!(p->nu_s > 0)) return fail(VLB_E_INVALID_ARG, "nu_s must be > 0 (tau_s1 > 1/2)");
    if (!(p->kappa > 0)) return fail(VLB_E_INVALID_ARG, "kappa must be > 0 (tau_p1 > 1/2)");
    if (!(p->lambda > 0)) return fail(VLB_E_INVALID_ARG, "lambda must be > 0");
    if (!(p->eta_p >= 0)) return fail(VLB_E_INVALID_ARG, "eta_p must be >= 0");
    if (!(p->Lambda_s > 0) || !(p->Lambda_p > 0))
        return fail(VLB_E_INVALID_ARG, "magic parameters must be > 0");
    if (p->flags & ~(VLB_FLAG_NO_SOURCE | VLB_FLAG_CURVED_YLW | VLB_FLAG_OPEN_NEBB))
        return fail(VLB_E_INVALID_ARG, "unknown flag");
    if ((p->flags & VLB_FLAG_OPEN_NEBB) && s->xmode != VLB_OPEN)
        return fail(VLB_E_UNSUPPORTED, "VLB_FLAG_OPEN_NEBB needs xmode = VLB_OPEN");
    if (p->model < VLB_OLDROYD_B || p->model > VLB_FENE_P)
        return fail(VLB_E_INVALID_ARG, "unknown constitutive model");
    if (p->model != VLB_OLDROYD_B && !std::isfinite(p->model_param))
        return fail(VLB_E_INVALID_ARG, "non-finite model parameter");
    if (p->model == VLB_GIESEKUS && !(p->model_param >= 0.0 && p->model_param <= 1.0))
        return fail(VLB_E_INVALID_ARG, "Giesekus alpha must lie in [0, 1]");
    if ((p->model == VLB_LPTT || p->model == VLB_EPTT) && !(p->model_param >= 0.0))
        return fail(VLB_E_INVALID_ARG, "PTT epsilon must be >= 0");
    if (p->model == VLB_FENE_P && !(p->model_param > 2.0))
        return fail(VLB_E_INVALID_ARG, "FENE-P L^2 must be > 2");
    s->params = *p;
    s->params_set = true;
    if (s->bound) return upload_run(s);
    return VLB_OK;
}

int vlb_set_force_field(vlb_sim* s, const void* fx, const void* fy) {
    int rc = check_bound(s);
    if (rc) return rc;
    if ((fx == nullptr) != (fy == nullptr))
        return fail(VLB_E_INVALID_ARG, "force field needs both components or neither");
    if (!fx) {
        s->force_field = false;
    } else {
        const size_t row = (size_t)s->nx * s->esz, dp = (size_t)s->pitch * s->esz;
        char* f0 = s->ws + s->off_force + (size_t)s->off0 * s->esz;
        VLB_HIP(hipMemcpy2DAsync(f0, dp, fx, row, row, s->ny, hipMemcpyDeviceToDevice, s->stream));
        VLB_HIP(hipMemcpy2DAsync(f0 + (size_t)s->plane * s->esz, dp, fy, row, row, s->ny,
                                 hipMemcpyDeviceToDevice, s->stream));
        s->force_field = true;
    }
    if (s->params_set) return upload_run(s);
    return VLB_OK;
}

int vlb_set_inlet(vlb_sim* s, const double* ux, const double* axx, const double* axy,
                  const double* ayy) {
    if (!s || !ux || !axx || !axy || !ayy) return fail(VLB_E_INVALID_ARG, "null argument");
    if (s->xmode != VLB_OPEN) return fail(VLB_E_UNSUPPORTED, "inlet needs xmode = VLB_OPEN");
    const double* src[4] = {ux, axx, axy, ayy};
    for (int c = 0; c < 4; ++c)
        for (int y = 0; y < s->ny; ++y) {
            if (!std::isfinite(src[c][y])) return fail(VLB_E_INVALID_ARG, "non-finite inlet value");
            s->inlet[(size_t)c * s->ny + y] = src[c][y];
        }
    if (!s->bound) return VLB_OK;
    VLB_HIP(hipMemcpyAsync(s->ws + s->off_inlet, s->inlet.data(), s->inlet.size() * sizeof(double),
                           hipMemcpyHostToDevice, s->stream));
    VLB_HIP(hipStreamSynchronize(s->stream));
    return VLB_OK;
}

int vlb_init_equilibrium(vlb_sim* s, const void* rho, const void* ux, const void* uy,
                         const void* axx, const void* axy, const void* ayy) {
    int rc = check_bound(s);
    if (rc) return rc;
    if (!s->params_set) return fail(VLB_E_STATE, "parameters not set (vlb_set_params)");
    if (s->prec == VLB_FP32) {
        VLB_HIP(vlb::launch_init<float>(make_run<float>(s), s->dptr<Run<float>>(s->off_run),
                                        (const float*)rho, (const float*)ux, (const float*)uy,
                                        (const float*)axx, (const float*)axy, (const float*)ayy,
                                        s->stream));
    } else {
        VLB_HIP(vlb::launch_init<double>(make_run<double>(s), s->dptr<Run<double>>(s->off_run),
                                         (const double*)rho, (const double*)ux, (const double*)uy,
                                         (const double*)axx, (const double*)axy,
                                         (const double*)ayy, s->stream));
    }
    VLB_HIP(vlb::launch_fill_bytes(s->ws + s->off_usnap, 2 * (size_t)s->nx * s->ny * s->esz, 0,
                                   s->stream));
    s->parity = 0;
    s->first = 1;
    s->step = 0;
    s->inited = true;
    return VLB_OK;
}

int vlb_step(vlb_sim* s, int64_t n) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (n < 0) return fail(VLB_E_INVALID_ARG, "negative step count");
    Range r("vlb_step");
    return s->prec == VLB_FP32 ? do_step<float>(s, n) : do_step<double>(s, n);
}

int vlb_get_step(const vlb_sim* s, int64_t* step) {
    if (!s || !step) return fail(VLB_E_INVALID_ARG, "null argument");
    *step = s->step;
    return VLB_OK;
}

int vlb_read_fields(vlb_sim* s, void* rho, void* ux, void* uy, void* axx, void* axy, void* ayy) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (s->prec == VLB_FP32) {
        VLB_HIP(vlb::launch_read<float>(make_run<float>(s), s->dptr<Run<float>>(s->off_run),
                                        s->parity, s->first, (float*)rho, (float*)ux, (float*)uy,
                                        (float*)axx, (float*)axy, (float*)ayy, s->stream));
    } else {
        VLB_HIP(vlb::launch_read<double>(make_run<double>(s), s->dptr<Run<double>>(s->off_run),
                                         s->parity, s->first, (double*)rho, (double*)ux,
                                         (double*)uy, (double*)axx, (double*)axy, (double*)ayy,
                                         s->stream));
    }
    return VLB_OK;
}

int vlb_read_history(vlb_sim* s, void* sxx, void* sxy, void* syy, void* uxp, void* uyp) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (s->prec == VLB_FP32)
        VLB_HIP(vlb::launch_read_history<float>(make_run<float>(s), s->dptr<Run<float>>(s->off_run),
                                                (float*)sxx, (float*)sxy, (float*)syy,
                                                (float*)uxp, (float*)uyp, s->stream));
    else
        VLB_HIP(vlb::launch_read_history<double>(make_run<double>(s), s->dptr<Run<double>>(s->off_run),
                                                 (double*)sxx, (double*)sxy, (double*)syy,
                                                 (double*)uxp, (double*)uyp, s->stream));
    return VLB_OK;
}

int vlb_monitors(vlb_sim* s, vlb_monitor* out) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!out) return fail(VLB_E_INVALID_ARG, "null output");
    vlb::MonitorAcc* acc = s->dptr<vlb::MonitorAcc>(s->off_mon);
    double* part = s->dptr<double>(s->off_monpart);
    if (s->prec == VLB_FP32) {
        VLB_HIP(vlb::launch_monitor<float>(make_run<float>(s), s->dptr<Run<float>>(s->off_run),
                                           s->parity, s->first, s->dptr<float>(s->off_usnap), part,
                                           acc, s->stream));
    } else {
        VLB_HIP(vlb::launch_monitor<double>(make_run<double>(s), s->dptr<Run<double>>(s->off_run),
                                            s->parity, s->first, s->dptr<double>(s->off_usnap),
                                            part, acc, s->stream));
    }
    vlb::MonitorAcc h{};
    VLB_HIP(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    VLB_HIP(hipStreamSynchronize(s->stream));
    for (int c = 0; c < 4; ++c) out->mass[c] = h.mass[c];
    out->residual = h.residual;
    out->umax = h.umax;
    out->step = s->step;
    out->nonfinite = (int64_t)h.nonfinite;
    out->spd_violations = (int64_t)h.spd;
    if (h.nonfinite) return fail(VLB_E_NONFINITE, "non-finite fields at step " + std::to_string(s->step));
    return VLB_OK;
}

int vlb_drag(vlb_sim* s, int circle, double* fx, double* fy) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!fx || !fy) return fail(VLB_E_INVALID_ARG, "null output");
    if (s->first) return fail(VLB_E_STATE, "the drag needs at least one step");
    if (circle >= (int)(s->circles.size() / 3)) return fail(VLB_E_INVALID_ARG, "no such circle");
    if (circle < 0 && s->ymode == VLB_WET)
        return fail(VLB_E_UNSUPPORTED, "the drag on wet-node walls is not built (circles only)");
    const int nl = (int)s->links.size();
    const int nb = (nl + 255) / 256;
    double* part = s->dptr<double>(s->off_dragpart);
    if (s->prec == VLB_FP32)
        VLB_HIP(vlb::launch_drag<float>(s->dptr<Run<float>>(s->off_run), s->dptr<int>(s->off_drag), nl,
                                        circle, s->parity, part, s->stream));
    else
        VLB_HIP(vlb::launch_drag<double>(s->dptr<Run<double>>(s->off_run), s->dptr<int>(s->off_drag),
                                         nl, circle, s->parity, part, s->stream));
    std::vector<double> h(2 * (size_t)std::max(1, nb), 0.0);
    if (nb > 0)
        VLB_HIP(hipMemcpyAsync(h.data(), part, 2 * (size_t)nb * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream));
    VLB_HIP(hipStreamSynchronize(s->stream));
    double sx = 0.0, sy = 0.0;
    for (int b = 0; b < nb; ++b) {
        sx += h[2 * b];
        sy += h[2 * b + 1];
    }
    *fx = sx;
    *fy = sy;
    return VLB_OK;
}

int vlb_state_bytes(const vlb_sim* s, size_t* bytes) {
    if (!s || !bytes) return fail(VLB_E_INVALID_ARG, "null argument");
    *bytes = 256 + 41 * (size_t)s->plane * s->esz;
    return VLB_OK;
}

static const unsigned long long kStateMagic = 0x564C425354415445ULL;  // "VLBSTATE"

// Header word 3 of a saved state: nx (bits 32-55), ny (bits 0-23), precision (bit 56),
// x and y boundary modes (bits 58-59, 60-61).  A state loads only into a simulation
// with the same word: the same plane layout, storage type and ghost-slot meaning.
static unsigned long long state_shape(const vlb_sim* s) {
    return ((unsigned long long)(unsigned)s->nx << 32) | (unsigned long long)(unsigned)s->ny |
           ((unsigned long long)(s->prec & 1) << 56) | ((unsigned long long)(s->xmode & 3) << 58) |
           ((unsigned long long)(s->ymode & 3) << 60);
}

int vlb_save_state(vlb_sim* s, void* dev, size_t bytes) {
    int rc = check_ready(s);
    if (rc) return rc;
    size_t need = 0;
    vlb_state_bytes(s, &need);
    if (!dev || bytes < need) return fail(VLB_E_WORKSPACE, "state buffer too small");
    char* d = static_cast<char*>(dev);
    VLB_HIP(vlb::launch_write_words(reinterpret_cast<unsigned long long*>(d), kStateMagic,
                                    (unsigned long long)s->step, (unsigned long long)s->first,
                                    state_shape(s), s->stream));
    const size_t pb = (size_t)s->plane * s->esz;
    VLB_HIP(hipMemcpyAsync(d + 256, s->ws + s->off_pop[s->parity], 36 * pb,
                           hipMemcpyDeviceToDevice, s->stream));
    VLB_HIP(hipMemcpyAsync(d + 256 + 36 * pb, s->ws + s->off_hist, 5 * pb,
                           hipMemcpyDeviceToDevice, s->stream));
    return VLB_OK;
}

int vlb_load_state(vlb_sim* s, const void* dev, size_t bytes) {
    int rc = check_bound(s);
    if (rc) return rc;
    if (!s->params_set) return fail(VLB_E_STATE, "parameters not set (vlb_set_params)");
    size_t need = 0;
    vlb_state_bytes(s, &need);
    if (!dev || bytes < need) return fail(VLB_E_WORKSPACE, "state buffer too small");
    unsigned long long hdr[4] = {0, 0, 0, 0};
    VLB_HIP(hipMemcpyAsync(hdr, dev, sizeof(hdr), hipMemcpyDeviceToHost, s->stream));
    VLB_HIP(hipStreamSynchronize(s->stream));
    if (hdr[0] != kStateMagic)
        return fail(VLB_E_INVALID_ARG, "state buffer does not hold a saved state");
    if (hdr[3] != state_shape(s))
        return fail(VLB_E_INVALID_ARG, "saved state is of another grid, precision or boundary kind");
    const char* d = static_cast<const char*>(dev);
    const size_t pb = (size_t)s->plane * s->esz;
    VLB_HIP(hipMemcpyAsync(s->ws + s->off_pop[0], d + 256, 36 * pb, hipMemcpyDeviceToDevice,
                           s->stream));
    VLB_HIP(hipMemcpyAsync(s->ws + s->off_hist, d + 256 + 36 * pb, 5 * pb,
                           hipMemcpyDeviceToDevice, s->stream));
    s->parity = 0;
    s->first = hdr[2] ? 1 : 0;
    s->step = (int64_t)hdr[1];
    s->inited = true;
    return VLB_OK;
}

int vlb_set_tile(vlb_sim* s, int ty) {
    if (!s) return fail(VLB_E_INVALID_ARG, "null simulation");
    if (ty != 1 && ty != 2 && ty != 4 && ty != 8) return fail(VLB_E_INVALID_ARG, "ty must be 1, 2, 4 or 8");
    s->ty = ty;
    drop_graphs(s);
    if (s->bound) return upload_items(s);
    return VLB_OK;
}

int vlb_set_schedule(vlb_sim* s, int tile_order, int waves) {
    if (!s) return fail(VLB_E_INVALID_ARG, "null simulation");
    if (tile_order < 0 || tile_order > 3) return fail(VLB_E_INVALID_ARG, "tile order must be 0 ... 3");
    if (waves != 0 && waves != 3 && waves != 4) return fail(VLB_E_INVALID_ARG, "waves must be 0, 3 or 4");
    s->sched_order = tile_order;
    s->sched_waves = waves;
    drop_graphs(s);
    if (s->bound) return upload_items(s);
    return VLB_OK;
}

}  // extern "C"

// ---- adjoint (periodic domains) ------------------------------------------------------

namespace {

template <class V>
__global__ void k_store_value(V v, V* dst) {
    if (threadIdx.x == 0) *dst = v;
}

struct AdjLayout {
    size_t state = 0;  // bytes of one saved state (vlb_save_state layout), 256-aligned
    int K = 1, nseg = 0;
    size_t off_desc = 0, off_adjdev = 0, off_ckpt = 0, off_slot = 0, off_a[2] = {0, 0},
           off_scr[2] = {0, 0}, off_gF = 0, off_part = 0, off_loss = 0, total = 0;
};

AdjLayout adj_layout(const vlb_sim* s, int64_t nsteps, int stride) {
    AdjLayout L;
    L.K = stride;
    L.nseg = (int)((nsteps + stride - 1) / stride);
    L.state = align256(256 + 41 * (size_t)s->plane * s->esz);
    const size_t pb = (size_t)s->plane * s->esz;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + bytes); return r; };
    const size_t rsz = s->prec == VLB_FP32 ? sizeof(Run<float>) : sizeof(Run<double>);
    const size_t asz = s->prec == VLB_FP32 ? sizeof(vlb::AdjDev<float>) : sizeof(vlb::AdjDev<double>);
    L.off_desc = take((size_t)L.K * rsz);
    L.off_adjdev = take(asz);
    L.off_ckpt = take((size_t)L.nseg * L.state);
    L.off_slot = take((size_t)L.K * L.state);
    L.off_a[0] = take(41 * pb);
    L.off_a[1] = take(41 * pb);
    // intermediates of consecutive reverse steps alternate between two buffers
    L.off_scr[0] = take(22 * pb);
    L.off_scr[1] = take(22 * pb);
    L.off_gF = take(2 * (size_t)s->plane * sizeof(double));
    L.off_part = take(2 * (size_t)std::max(1, s->nitems) * sizeof(double));
    L.off_loss = take((size_t)std::max(1, s->nitems) * sizeof(double));
    L.total = o;
    return L;
}

int adj_check(const vlb_sim* s, int64_t nsteps, int stride) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (s->xmode == VLB_OPEN || s->ymode == VLB_WET)
        return fail(VLB_E_UNSUPPORTED,
                    "the adjoint covers periodic axes, half-way walls and solid masks, not open "
                    "ends or wet-node walls");
    if (s->has_curved && (s->params.flags & VLB_FLAG_CURVED_YLW))
        return fail(VLB_E_UNSUPPORTED, "the adjoint covers linear interpolated bounce-back on "
                                       "curved links, not VLB_FLAG_CURVED_YLW");
    if (nsteps < 0 || stride < 1) return fail(VLB_E_INVALID_ARG, "nsteps >= 0 and stride >= 1 required");
    return VLB_OK;
}

// Descriptor k of the recompute: reads state slot k, writes slot k + 1 (history too).
template <class T>
int adj_upload_desc(vlb_sim* s, const AdjLayout& L, char* ws) {
    const size_t pb = (size_t)s->plane * s->esz;
    Run<T>* d = reinterpret_cast<Run<T>*>(ws + L.off_desc);
    for (int k = 0; k < L.K; ++k) {
        char* sk = ws + L.off_slot + (size_t)k * L.state;
        char* sn = k + 1 < L.K ? sk + L.state : sk;
        Run<T> r = make_run<T>(s);
        r.pop[0] = reinterpret_cast<T*>(sk + 256);
        r.pop[1] = reinterpret_cast<T*>(sn + 256);
        r.hist = reinterpret_cast<T*>(sk + 256 + 36 * pb);
        r.hist_out = reinterpret_cast<T*>(sn + 256 + 36 * pb);
        hipLaunchKernelGGL((k_store_value<Run<T>>), dim3(1), dim3(64), 0, s->stream, r, d + k);
        VLB_HIP(hipGetLastError());
    }
    return VLB_OK;
}

template <class T>
int adj_forward(vlb_sim* s, int64_t nsteps, int stride, char* ws, size_t bytes) {
    const AdjLayout L = adj_layout(s, nsteps, stride);
    s->adj.valid = false;
    s->adj.ws = ws;
    s->adj.bytes = bytes;
    s->adj.nsteps = nsteps;
    s->adj.stride = stride;
    s->adj.step0 = s->step;
    s->adj.first0 = s->first;
    s->adj.ty = s->ty;
    for (int g = 0; g < L.nseg; ++g) {
        char* ck = ws + L.off_ckpt + (size_t)g * L.state;
        int rc = vlb_save_state(s, ck, L.state);
        if (rc) return rc;
        const int64_t len = std::min<int64_t>(stride, nsteps - (int64_t)g * stride);
        rc = do_step<T>(s, len);
        if (rc) return rc;
    }
    s->adj.version = s->version;
    s->adj.valid = true;
    return VLB_OK;
}

template <class T>
int adj_backward(vlb_sim* s, const void* gx, const void* gy, int is_target, double* loss,
                 double* dlam, double* deta, void* dFx, void* dFy) {
    const int64_t nsteps = s->adj.nsteps;
    const int stride = s->adj.stride;
    char* ws = s->adj.ws;
    const AdjLayout L = adj_layout(s, nsteps, stride);
    int rc = adj_upload_desc<T>(s, L, ws);
    if (rc) return rc;
    vlb::AdjDev<T> a{};
    a.nx = s->nx; a.ny = s->ny; a.pitch = s->pitch; a.off0 = s->off0; a.plane = s->plane;
    a.scr = nullptr;
    T* scr[2] = {reinterpret_cast<T*>(ws + L.off_scr[0]), reinterpret_cast<T*>(ws + L.off_scr[1])};
    a.gF = reinterpret_cast<double*>(ws + L.off_gF);
    a.part = reinterpret_cast<double*>(ws + L.off_part);
    a.lossp = reinterpret_cast<double*>(ws + L.off_loss);
    a.seed_x = static_cast<const T*>(gx);
    a.seed_y = static_cast<const T*>(gy);
    a.seed_is_target = is_target;
    size_t nfluid = (size_t)s->nx * s->ny;
    if (!s->solid.empty()) nfluid -= (size_t)std::count(s->solid.begin(), s->solid.end(), 1);
    a.inv_nfluid = 1.0 / (double)std::max<size_t>(nfluid, 1);
    vlb::AdjDev<T>* ad = reinterpret_cast<vlb::AdjDev<T>*>(ws + L.off_adjdev);
    hipLaunchKernelGGL((k_store_value<vlb::AdjDev<T>>), dim3(1), dim3(64), 0, s->stream, a, ad);
    VLB_HIP(hipGetLastError());
    const vlb::Item* items = s->dptr<vlb::Item>(s->off_items);
    const vlb::FillItem* fill = s->dptr<vlb::FillItem>(s->off_fill_items);
    T* abuf[2] = {reinterpret_cast<T*>(ws + L.off_a[0]), reinterpret_cast<T*>(ws + L.off_a[1])};
    const Run<T>* rs = s->dptr<Run<T>>(s->off_run);
    VLB_HIP(vlb::launch_adj_seed<T>(rs, ad, items, s->nitems, s->ty, s->dptr<T>(s->off_pop[s->parity]),
                                    s->first ? 0 : 1, abuf[0], s->stream));
    int cur = 0, sc = 0, fused = 0;
    const Run<T>* desc = reinterpret_cast<const Run<T>*>(ws + L.off_desc);
    for (int g = L.nseg - 1; g >= 0; --g) {
        const int64_t len = std::min<int64_t>(stride, nsteps - (int64_t)g * stride);
        VLB_HIP(hipMemcpyAsync(ws + L.off_slot, ws + L.off_ckpt + (size_t)g * L.state, L.state,
                               hipMemcpyDeviceToDevice, s->stream));
        for (int64_t k = 0; k + 1 < len; ++k) {
            const int first = (g == 0 && k == 0 && s->adj.first0) ? 1 : 0;
            VLB_HIP(vlb::launch_step<T>(desc + k, items, s->nitems, s->ty, 0, first, 0,
                                        step_waves(s->sched_waves, resident_state(s)), s->stream));
            VLB_HIP(vlb::launch_fill<T>(desc + k, fill, (int)s->fill_items.size(), 1, s->stream));
        }
        for (int64_t k = len - 1; k >= 0; --k) {
            const int first = (g == 0 && k == 0 && s->adj.first0) ? 1 : 0;
            // the later step's gather runs inside this launch (all but the first)
            VLB_HIP(vlb::launch_adj_step<T>(desc + k, ad, items, s->nitems, s->ty, first,
                                            s->has_bits ? 1 : 0, fused, abuf[cur],
                                            abuf[cur ^ 1], scr[sc], scr[sc ^ 1], s->stream));
            cur ^= 1;
            sc ^= 1;
            fused = 1;
        }
    }
    if (fused)
        VLB_HIP(vlb::launch_adj_gather<T>(rs, ad, items, s->nitems, s->ty, s->has_bits ? 1 : 0,
                                          scr[sc], abuf[cur], s->stream));
    const size_t row = (size_t)s->nx * sizeof(double);
    const size_t pitchb = (size_t)s->pitch * sizeof(double);
    const double* gF = reinterpret_cast<const double*>(ws + L.off_gF) + s->off0;
    if (dFx) VLB_HIP(hipMemcpy2DAsync(dFx, row, gF, pitchb, row, s->ny, hipMemcpyDeviceToDevice, s->stream));
    if (dFy) VLB_HIP(hipMemcpy2DAsync(dFy, row, gF + s->plane, pitchb, row, s->ny, hipMemcpyDeviceToDevice, s->stream));
    std::vector<double> part(2 * (size_t)s->nitems), lossp((size_t)s->nitems);
    VLB_HIP(hipMemcpyAsync(part.data(), ws + L.off_part, part.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream));
    VLB_HIP(hipMemcpyAsync(lossp.data(), ws + L.off_loss, lossp.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream));
    VLB_HIP(hipStreamSynchronize(s->stream));
    double sl = 0.0, se = 0.0, sloss = 0.0;
    for (int b = 0; b < s->nitems; ++b) {
        sl += part[2 * b];
        se += part[2 * b + 1];
        sloss += lossp[b];
    }
    if (dlam) *dlam = sl;
    if (deta) *deta = se;
    if (loss) *loss = is_target ? sloss : 0.0;
    return VLB_OK;
}

int adj_ws_check(const vlb_sim* s, int64_t nsteps, int stride, void* ws, size_t bytes) {
    const AdjLayout L = adj_layout(s, nsteps, stride);
    if (!ws || ((uintptr_t)ws & 255u) || bytes < L.total)
        return fail(VLB_E_WORKSPACE, "adjoint workspace missing, misaligned or smaller than " +
                                         std::to_string(L.total) + " bytes");
    return VLB_OK;
}

}  // namespace

extern "C" {

int vlb_params_from_groups(double Re, double Wi, double beta, double Sc, double Ma, double Lc,
                           double Lambda_s, double Lambda_p, vlb_params* out, double* uc) {
    if (!out) return fail(VLB_E_INVALID_ARG, "null output");
    if (!(Re > 0) || !(Wi > 0) || !(Sc > 0) || !(Ma > 0) || !(Lc > 0) || !(Lambda_s > 0) ||
        !(Lambda_p > 0) || !(beta > 0) || !(beta <= 1))
        return fail(VLB_E_INVALID_ARG, "groups must be positive and 0 < beta <= 1");
    const double Uc = Ma * std::sqrt(1.0 / 3.0);
    const double nu0 = Uc * Lc / Re;
    vlb_params p{};
    p.nu_s = beta * nu0;
    p.eta_p = (1.0 - beta) * nu0;
    p.lambda = Wi * Lc / Uc;
    p.kappa = p.nu_s / Sc;
    p.Lambda_s = Lambda_s;
    p.Lambda_p = Lambda_p;
    *out = p;
    if (uc) *uc = Uc;
    return VLB_OK;
}

int vlb_adjoint_workspace_bytes(const vlb_sim* s, int64_t nsteps, int stride, size_t* bytes) {
    if (!s || !bytes) return fail(VLB_E_INVALID_ARG, "null argument");
    if (nsteps < 0 || stride < 1) return fail(VLB_E_INVALID_ARG, "nsteps >= 0 and stride >= 1 required");
    *bytes = adj_layout(s, nsteps, stride).total;
    return VLB_OK;
}

int vlb_adjoint_forward(vlb_sim* s, int64_t nsteps, int stride, void* ws, size_t bytes) {
    int rc = adj_check(s, nsteps, stride);
    if (rc) return rc;
    rc = adj_ws_check(s, nsteps, stride, ws, bytes);
    if (rc) return rc;
    char* w = static_cast<char*>(ws);
    Range r("vlb_adjoint_forward");
    return s->prec == VLB_FP32 ? adj_forward<float>(s, nsteps, stride, w, bytes)
                               : adj_forward<double>(s, nsteps, stride, w, bytes);
}

static int adj_backward_checked(vlb_sim* s, const void* gx, const void* gy, int is_target,
                                double* loss, double* dlam, double* deta, void* dFx, void* dFy,
                                void* ws, size_t bytes) {
    int rc = adj_check(s, 0, 1);
    if (rc) return rc;
    if (!gx || !gy) return fail(VLB_E_INVALID_ARG, "null velocity seed");
    if (!s->adj.valid || s->adj.ws != ws || s->adj.bytes != bytes)
        return fail(VLB_E_STATE, "no vlb_adjoint_forward recorded in this workspace");
    if (s->step != s->adj.step0 + s->adj.nsteps || s->adj.version != s->version ||
        s->ty != s->adj.ty)
        return fail(VLB_E_STATE, "simulation changed since vlb_adjoint_forward");
    Range r("vlb_adjoint_backward");
    return s->prec == VLB_FP32
               ? adj_backward<float>(s, gx, gy, is_target, loss, dlam, deta, dFx, dFy)
               : adj_backward<double>(s, gx, gy, is_target, loss, dlam, deta, dFx, dFy);
}

int vlb_adjoint_backward(vlb_sim* s, const void* dL_dux, const void* dL_duy, double* dL_dlambda,
                         double* dL_detap, void* dL_dFx, void* dL_dFy, void* ws, size_t bytes) {
    return adj_backward_checked(s, dL_dux, dL_duy, 0, nullptr, dL_dlambda, dL_detap, dL_dFx,
                                dL_dFy, ws, bytes);
}

int vlb_adjoint(vlb_sim* s, int64_t nsteps, int stride, const void* ux_tgt, const void* uy_tgt,
                double* loss, double* dL_dlambda, double* dL_detap, void* dL_dFx, void* dL_dFy,
                void* ws, size_t bytes) {
    if (!ux_tgt || !uy_tgt) return fail(VLB_E_INVALID_ARG, "null target velocity");
    int rc = vlb_adjoint_forward(s, nsteps, stride, ws, bytes);
    if (rc) return rc;
    return adj_backward_checked(s, ux_tgt, uy_tgt, 1, loss, dL_dlambda, dL_detap, dL_dFx, dL_dFy,
                                ws, bytes);
}

}  // extern "C"

// ---- batches --------------------------------------------------------------------

namespace {

void batch_layout(vlb_batch* b) {
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + bytes); return r; };
    const size_t rsz = b->prec == VLB_FP32 ? sizeof(Run<float>) : sizeof(Run<double>);
    b->off_runs = take(b->sims.size() * rsz);
    b->off_items = take(std::max<size_t>(1, b->items.size()) * sizeof(vlb::Item));
    b->off_fill_items = take(std::max<size_t>(1, b->fill_items.size()) * sizeof(vlb::FillItem));
    b->off_queues = take(2 * vlb::kBatchQueues * sizeof(int));  // persistent form's counters
    b->total = o;
}

int batch_lists(vlb_batch* b, vlb_sim* const* sims, int n, int ty) {
    if (!sims || n < 1) return fail(VLB_E_INVALID_ARG, "batch needs at least one simulation");
    if (ty != 1 && ty != 2 && ty != 4 && ty != 8) return fail(VLB_E_INVALID_ARG, "ty must be 1, 2, 4 or 8");
    b->sims.assign(sims, sims + n);
    b->ty = ty;
    b->prec = sims[0]->prec;
    double state_bytes = 0;
    std::vector<vlb::Item>& tiles = b->tiles;
    tiles.clear();
    for (int r = 0; r < n; ++r) {
        const vlb_sim* s = sims[r];
        if (!s) return fail(VLB_E_INVALID_ARG, "null simulation in batch");
        if (s->prec != b->prec) return fail(VLB_E_INVALID_ARG, "batch mixes precisions");
        // a member listed twice would be advanced twice per batch step (its buffer
        // parity flipped twice), so later reads would see the stale buffer
        for (int q = 0; q < r; ++q)
            if (sims[q] == s) return fail(VLB_E_INVALID_ARG, "simulation listed twice in batch");
        const int ntx = (s->nx + 63) / 64, nty = (s->ny + ty - 1) / ty;
        for (int t = 0; t < ntx * nty; ++t) tiles.push_back(vlb::Item{r, t % ntx, t / ntx, 0});
        for (const vlb::FillItem& fi : s->fill_items)
            b->fill_items.push_back(vlb::FillItem{r, fi.first, fi.count, 0});
        state_bytes += 2.0 * 36.0 * (double)s->nx * (double)s->ny * (double)s->esz;
    }
    // the concatenated tiles in the order of the schedule (as for a single run)
    b->resident = state_bytes <= 192.0 * 1024 * 1024;
    b->streaming = b->resident ? 0 : 1;
    order_tiles(tiles, effective_order(b->sched_order, b->resident), b->items);
    batch_layout(b);
    return VLB_OK;
}

// Copies member r's descriptor into the batch's array, ordered on the shared stream.
template <class T>
int batch_store_run(vlb_batch* b, int r) {
    Run<T>* dst = reinterpret_cast<Run<T>*>(b->ws + b->off_runs) + r;
    hipLaunchKernelGGL((k_store_run<T>), dim3(1), dim3(64), 0, b->stream, make_run<T>(b->sims[r]), dst);
    VLB_HIP(hipGetLastError());
    b->versions[r] = b->sims[r]->version;
    return VLB_OK;
}

template <class T>
int batch_upload(vlb_batch* b) {
    b->versions.assign(b->sims.size(), 0);
    for (int r = 0; r < (int)b->sims.size(); ++r) {
        int rc = batch_store_run<T>(b, r);
        if (rc) return rc;
    }
    VLB_HIP(hipMemcpyAsync(b->ws + b->off_items, b->items.data(), b->items.size() * sizeof(vlb::Item),
                           hipMemcpyHostToDevice, b->stream));
    VLB_HIP(vlb::launch_fill_bytes(b->ws + b->off_queues, 2 * vlb::kBatchQueues * sizeof(int), 0,
                                   b->stream));
    if (!b->fill_items.empty())
        VLB_HIP(hipMemcpyAsync(b->ws + b->off_fill_items, b->fill_items.data(),
                               b->fill_items.size() * sizeof(vlb::FillItem), hipMemcpyHostToDevice,
                               b->stream));
    VLB_HIP(hipStreamSynchronize(b->stream));
    return VLB_OK;
}

// Re-copies the descriptors of members whose parameters, force or inlet changed.
template <class T>
int batch_refresh(vlb_batch* b) {
    for (int r = 0; r < (int)b->sims.size(); ++r)
        if (b->versions[r] != b->sims[r]->version) {
            int rc = batch_store_run<T>(b, r);
            if (rc) return rc;
        }
    return VLB_OK;
}

void batch_drop_graphs(vlb_batch* b) {
    for (auto& g : b->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Steps per cooperative launch of the persistent batch kernel.
constexpr int64_t kPersistentChunk = 256;

template <class T>
int batch_launch(vlb_batch* b, int par, int first) {
    const Run<T>* rd = reinterpret_cast<const Run<T>*>(b->ws + b->off_runs);
    const vlb::Item* it = reinterpret_cast<const vlb::Item*>(b->ws + b->off_items);
    const vlb::FillItem* fi = reinterpret_cast<const vlb::FillItem*>(b->ws + b->off_fill_items);
    VLB_HIP(vlb::launch_step<T>(rd, it, (int)b->items.size(), b->ty, par, first, b->streaming,
                                step_waves(b->sched_waves, b->resident), b->stream));
    VLB_HIP(vlb::launch_fill<T>(rd, fi, (int)b->fill_items.size(), par ^ 1, b->stream));
    return VLB_OK;
}

template <class T>
int batch_step(vlb_batch* b, int64_t n) {
    int rc0 = batch_refresh<T>(b);
    if (rc0) return rc0;
    vlb_sim* s0 = b->sims[0];
    auto advance = [&](int64_t k) {
        b->step += k;
        for (vlb_sim* s : b->sims) {
            s->step += k;
            if (k % 2) s->parity ^= 1;
            if (k > 0) s->first = 0;
        }
    };
    if (b->persistent) {
        // one cooperative launch per chunk of at most kPersistentChunk steps (bounded
        // kernel duration); the first step of the members is the chunk's first
        const Run<T>* rd = reinterpret_cast<const Run<T>*>(b->ws + b->off_runs);
        const vlb::Item* it = reinterpret_cast<const vlb::Item*>(b->ws + b->off_items);
        const vlb::FillItem* fi = reinterpret_cast<const vlb::FillItem*>(b->ws + b->off_fill_items);
        while (n > 0) {
            const int k = (int)std::min<int64_t>(n, kPersistentChunk);
            VLB_HIP(vlb::launch_batch<T>(rd, it, (int)b->items.size(), fi, (int)b->fill_items.size(),
                                         k, b->ty, s0->parity, s0->first, b->streaming,
                                         reinterpret_cast<int*>(b->ws + b->off_queues), b->stream));
            advance(k);
            n -= k;
        }
        return VLB_OK;
    }
    if (s0->first && n > 0) {
        int rc = batch_launch<T>(b, s0->parity, 1);
        if (rc) return rc;
        advance(1);
        --n;
    }
    if (b->graph_chunk > 0 && b->stream != nullptr) {
        const int64_t per = 2 * (int64_t)b->graph_chunk;
        while (n >= per) {
            const int par = s0->parity;
            if (!b->graph[par]) {
                hipGraph_t g = nullptr;
                VLB_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                int rc = VLB_OK;
                int p = par;
                for (int k = 0; k < per && rc == VLB_OK; ++k) {
                    rc = batch_launch<T>(b, p, 0);
                    p ^= 1;
                }
                hipError_t e2 = hipStreamEndCapture(b->stream, &g);
                if (rc || e2 != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc ? rc : fail(VLB_E_HIP, std::string("batch graph capture: ") + hipGetErrorString(e2));
                }
                hipError_t e3 = hipGraphInstantiate(&b->graph[par], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e3 != hipSuccess) return fail(VLB_E_HIP, std::string("batch graph: ") + hipGetErrorString(e3));
            }
            VLB_HIP(hipGraphLaunch(b->graph[par], b->stream));
            advance(per);
            n -= per;
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        int rc = batch_launch<T>(b, s0->parity, 0);
        if (rc) return rc;
        advance(1);
    }
    return VLB_OK;
}

}  // namespace

// Static scratch of vlb_batch_create_noalloc: the work lists, member descriptors and
// persistent-form counters of one batch per device, in a file-scope device array that
// each device holds for the life of the process.  Host code never uses the array's name
// as an address (it is a host-side stand-in): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kBatchScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kBatchScratchBytes];

namespace {

struct ScratchSlot {
    void* ptr = nullptr;  // device address of `scratch` on this device
    bool busy = false;    // a live noalloc batch holds it
};
std::mutex g_scratch_mu;
std::map<int, ScratchSlot> g_scratch;

// Member checks shared by both batch constructors.
int batch_check_members(const vlb_batch* b, vlb_sim* const* sims) {
    for (vlb_sim* s : b->sims) {
        int rc = check_ready(s);
        if (rc) return rc;
        if (s->stream != sims[0]->stream) return fail(VLB_E_INVALID_ARG, "batch members must share one stream");
        if (s->step != sims[0]->step || s->parity != sims[0]->parity || s->first != sims[0]->first)
            return fail(VLB_E_STATE, "batch members must be at the same step");
    }
    return VLB_OK;
}

void batch_release_scratch(vlb_batch* b) {
    if (b->scratch_dev < 0) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    g_scratch[b->scratch_dev].busy = false;
    b->scratch_dev = -1;
}

}  // namespace

extern "C" {

int vlb_batch_workspace_bytes(vlb_sim* const* sims, int n, int ty, size_t* bytes) {
    if (!bytes) return fail(VLB_E_INVALID_ARG, "null output");
    vlb_batch tmp;
    int rc = batch_lists(&tmp, sims, n, ty);
    if (rc) return rc;
    *bytes = tmp.total;
    return VLB_OK;
}

int vlb_batch_create(vlb_sim* const* sims, int n, int ty, void* ws, size_t bytes, vlb_batch** out) {
    if (!out) return fail(VLB_E_INVALID_ARG, "null output");
    *out = nullptr;
    vlb_batch* b = new (std::nothrow) vlb_batch();
    if (!b) return fail(VLB_E_INVALID_ARG, "out of host memory");
    int rc = batch_lists(b, sims, n, ty);
    if (rc) { delete b; return rc; }
    rc = batch_check_members(b, sims);
    if (rc) { delete b; return rc; }
    if (!ws || ((uintptr_t)ws & 255u) || bytes < b->total) {
        delete b;
        return fail(VLB_E_WORKSPACE, "batch workspace missing, misaligned or smaller than " +
                                         std::to_string(b->total) + " bytes");
    }
    b->ws = static_cast<char*>(ws);
    b->bytes = bytes;
    b->stream = sims[0]->stream;
    b->step = sims[0]->step;
    rc = b->prec == VLB_FP32 ? batch_upload<float>(b) : batch_upload<double>(b);
    if (rc) { delete b; return rc; }
    *out = b;
    return VLB_OK;
}

int vlb_batch_create_noalloc(vlb_sim* const* sims, int n, int ty, vlb_batch** out) {
    if (!out) return fail(VLB_E_INVALID_ARG, "null output");
    *out = nullptr;
    vlb_batch* b = new (std::nothrow) vlb_batch();
    if (!b) return fail(VLB_E_INVALID_ARG, "out of host memory");
    int rc = batch_lists(b, sims, n, ty);
    if (rc) { delete b; return rc; }
    if (b->total > kBatchScratchBytes) {
        const size_t need = b->total;
        delete b;
        return fail(VLB_E_WORKSPACE, "batch lists need " + std::to_string(need) +
                                         " bytes; the static scratch holds " +
                                         std::to_string(kBatchScratchBytes));
    }
    rc = batch_check_members(b, sims);
    if (rc) { delete b; return rc; }
    int dev = 0;
    {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) { delete b; return fail(VLB_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e)); }
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ScratchSlot& slot = g_scratch[dev];
        if (!slot.ptr) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                delete b;
                return fail(VLB_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            }
            slot.ptr = ptr;
        }
        if (slot.busy) {
            delete b;
            return fail(VLB_E_STATE, "the static batch scratch of this device is held by another "
                                     "batch (destroy it first)");
        }
        slot.busy = true;
        b->ws = static_cast<char*>(slot.ptr);
        b->scratch_dev = dev;
    }
    b->bytes = kBatchScratchBytes;
    b->stream = sims[0]->stream;
    b->step = sims[0]->step;
    rc = b->prec == VLB_FP32 ? batch_upload<float>(b) : batch_upload<double>(b);
    if (rc) { batch_release_scratch(b); delete b; return rc; }
    *out = b;
    return VLB_OK;
}

int vlb_batch_set_persistent(vlb_batch* b, int on) {
    if (!b) return fail(VLB_E_INVALID_ARG, "null batch");
    if (on != 0 && on != 1) return fail(VLB_E_INVALID_ARG, "persistent must be 0 or 1");
    if (on) {
        int dev = 0, coop = 0;
        VLB_HIP(hipGetDevice(&dev));
        VLB_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        if (!coop) return fail(VLB_E_UNSUPPORTED, "device has no cooperative launch");
    }
    b->persistent = on;
    return VLB_OK;
}

int vlb_batch_step(vlb_batch* b, int64_t n) {
    if (!b) return fail(VLB_E_INVALID_ARG, "null batch");
    if (n < 0) return fail(VLB_E_INVALID_ARG, "negative step count");
    for (vlb_sim* s : b->sims)
        if (s->step != b->step || s->parity != b->sims[0]->parity || s->first != b->sims[0]->first)
            return fail(VLB_E_STATE, "batch member was stepped or reloaded outside the batch");
    Range r("vlb_batch_step");
    return b->prec == VLB_FP32 ? batch_step<float>(b, n) : batch_step<double>(b, n);
}

int vlb_batch_read_fields(vlb_batch* b, int run, void* rho, void* ux, void* uy, void* axx,
                          void* axy, void* ayy) {
    if (!b || run < 0 || run >= (int)b->sims.size()) return fail(VLB_E_INVALID_ARG, "run index out of range");
    return vlb_read_fields(b->sims[run], rho, ux, uy, axx, axy, ayy);
}

int vlb_batch_set_graph_chunk(vlb_batch* b, int chunk) {
    if (!b || chunk < 0 || chunk > 4096) return fail(VLB_E_INVALID_ARG, "chunk out of range");
    batch_drop_graphs(b);
    b->graph_chunk = chunk;
    return VLB_OK;
}

int vlb_batch_set_schedule(vlb_batch* b, int tile_order, int waves) {
    if (!b) return fail(VLB_E_INVALID_ARG, "null batch");
    if (tile_order < 0 || tile_order > 3) return fail(VLB_E_INVALID_ARG, "tile order must be 0 ... 3");
    if (waves != 0 && waves != 3 && waves != 4) return fail(VLB_E_INVALID_ARG, "waves must be 0, 3 or 4");
    b->sched_order = tile_order;
    b->sched_waves = waves;
    batch_drop_graphs(b);
    order_tiles(b->tiles, effective_order(b->sched_order, b->resident), b->items);
    VLB_HIP(hipMemcpyAsync(b->ws + b->off_items, b->items.data(), b->items.size() * sizeof(vlb::Item),
                           hipMemcpyHostToDevice, b->stream));
    VLB_HIP(hipStreamSynchronize(b->stream));
    return VLB_OK;
}

void vlb_batch_destroy(vlb_batch* b) {
    if (!b) return;
    batch_drop_graphs(b);
    batch_release_scratch(b);
    delete b;
}

int vlb_set_store_mode(vlb_sim* s, int mode) {
    if (!s || mode < 0 || mode > 2) return fail(VLB_E_INVALID_ARG, "store mode must be 0, 1 or 2");
    s->store_mode = mode;
    drop_graphs(s);
    return VLB_OK;
}

int vlb_set_graph_chunk(vlb_sim* s, int chunk) {
    if (!s || chunk < 0 || chunk > 4096) return fail(VLB_E_INVALID_ARG, "chunk out of range");
    drop_graphs(s);
    s->graph_chunk = chunk;
    return VLB_OK;
}

}  // extern "C"
