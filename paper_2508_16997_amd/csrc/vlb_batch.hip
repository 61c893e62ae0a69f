// vlb_batch.hip -- persistent form of the batched step: one cooperative launch advances
// every run of a batch by up to a chunk of steps, with grid-wide barriers between the
// tiles of a step and its boundary fills.  The tile body is the one of the per-step
// kernel (vlb_step.h), so results are bit-identical to the per-step launches.
#include <algorithm>

#include <hip/hip_cooperative_groups.h>

#include "vlb_step.h"

namespace cg = cooperative_groups;

namespace vlb {
namespace {

// Persistent form for batches: one cooperative launch advances every run nsteps steps.
// The ordered item list is split into nq queues (item w belongs to queue w % nq;
// nq = 8 when the grid has at least 8 workgroups).  A workgroup first draws items --
// kBatchChunk consecutive entries per atomic -- of the queue of the XCD it runs on from
// that queue's atomic counter, so each XCD sweeps its band in order (neighbouring tiles, whose rows the
// pulls share, run at about the same time and meet in that XCD's L2) and faster
// workgroups take more tiles; then it helps drain the other queues, so every item is
// taken whatever the placement of the workgroups.  A grid-wide barrier separates the
// tiles of a step from its fill ops (dealt round-robin), and the fills from the next
// step.  Two counter sets alternate between steps; the set of step n + 1 is cleared
// during the fills of step n, when nobody draws from it, and the last one after the
// final barrier, so both are zero between launches.
// Consecutive queue entries a workgroup takes per atomic draw.
constexpr int kBatchChunk = 4;

template <class S, int TY, bool NT>
__global__ __launch_bounds__((StepBounds<S, TY, 3>::threads), (StepBounds<S, TY, 3>::batch_waves_per_eu)) void k_batch(
    const RunDev<S>* __restrict__ runs, const Item* __restrict__ items, int nitems,
    const FillItem* __restrict__ fitems, int nfitems, int nsteps, int parity, int first,
    int* __restrict__ queues) {
    cg::grid_group grid = cg::this_grid();
    __shared__ int s_next;
    const int tid = threadIdx.y * 64 + threadIdx.x;
    const int nq = gridDim.x < kBatchQueues ? (int)gridDim.x : kBatchQueues;
    unsigned xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
    const int q0 = (int)(xcc % (unsigned)nq);
    for (int n = 0; n < nsteps; ++n) {
        for (int j = 0; j < nq; ++j) {
            const int q = q0 + j < nq ? q0 + j : q0 + j - nq;
            const int qlen = (nitems - q + nq - 1) / nq;  // items q, q + nq, ...
            int* ctr = queues + (n & 1) * kBatchQueues + q;
            __syncthreads();  // every read of s_next is done
            if (tid == 0) s_next = atomicAdd(ctr, kBatchChunk);
            __syncthreads();
            int k = s_next;
            while (k < qlen) {
                // draw the following chunk now: the atomic's round trip overlaps this one
                int k_next = 0;
                if (tid == 0) k_next = atomicAdd(ctr, kBatchChunk);
                const int kend = min(k + kBatchChunk, qlen);
                for (int kk = k; kk < kend; ++kk) {
                    int lane0;
                    asm volatile("v_mov_b32 %0, 0" : "=v"(lane0));
                    step_tile<S, TY, NT>(runs, items[q + kk * nq], parity, first, lane0);
                    __syncthreads();  // this tile's LDS reads are done (and every read of s_next)
                }
                if (tid == 0) s_next = k_next;
                __syncthreads();
                k = s_next;
            }
        }
        grid.sync();
        if (blockIdx.x == 0 && tid < kBatchQueues)
            atomicExch(queues + ((n + 1) & 1) * kBatchQueues + tid, 0);
        parity ^= 1;
        first = 0;
        for (int w = blockIdx.x; w < nfitems; w += gridDim.x) {
            const FillItem fi = fitems[w];
            const RunDev<S>& R = runs[fi.run];
            for (int j = tid; j < fi.count; j += 64 * TY)
                apply_fill_op(R, R.fill[fi.first + j], R.pop[parity]);
        }
        grid.sync();
    }
    if (blockIdx.x == 0 && tid < kBatchQueues)
        atomicExch(queues + ((nsteps - 1) & 1) * kBatchQueues + tid, 0);
}

}  // namespace

template <class S, int TY, bool NT>
hipError_t launch_batch_ty(const RunDev<S>* runs_dev, const Item* items_dev, int nitems,
                           const FillItem* fitems_dev, int nfitems, int nsteps, int parity,
                           int first, int* queues, hipStream_t s) {
    auto kern = k_batch<S, TY, NT>;
    int per_cu = 0, dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * TY, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    // every workgroup must be resident at once for the grid barrier; more than the
    // work needs only adds barrier participants; a multiple of the 8 XCDs gives every
    // XCD the same number of workgroups
    int grid = std::min(nitems, per_cu * ncu);
    if (grid >= kBatchQueues) grid -= grid % kBatchQueues;
    grid = std::max(1, grid);
    void* args[] = {(void*)&runs_dev, (void*)&items_dev, (void*)&nitems, (void*)&fitems_dev,
                    (void*)&nfitems, (void*)&nsteps, (void*)&parity, (void*)&first,
                    (void*)&queues};
    return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(64, TY), args, 0, s);
}

template <class S, bool NT>
hipError_t launch_batch_nt(const RunDev<S>* runs_dev, const Item* items_dev, int nitems,
                           const FillItem* fitems_dev, int nfitems, int nsteps, int ty, int parity,
                           int first, int* queues, hipStream_t s) {
    switch (ty) {
        case 1: return launch_batch_ty<S, 1, NT>(runs_dev, items_dev, nitems, fitems_dev, nfitems, nsteps, parity, first, queues, s);
        case 2: return launch_batch_ty<S, 2, NT>(runs_dev, items_dev, nitems, fitems_dev, nfitems, nsteps, parity, first, queues, s);
        case 4: return launch_batch_ty<S, 4, NT>(runs_dev, items_dev, nitems, fitems_dev, nfitems, nsteps, parity, first, queues, s);
        case 8: return launch_batch_ty<S, 8, NT>(runs_dev, items_dev, nitems, fitems_dev, nfitems, nsteps, parity, first, queues, s);
        default: return hipErrorInvalidValue;
    }
}

template <class S>
hipError_t launch_batch(const RunDev<S>* runs_dev, const Item* items_dev, int nitems,
                        const FillItem* fitems_dev, int nfitems, int nsteps, int ty, int parity,
                        int first, int streaming, int* queues, hipStream_t s) {
    if (nitems <= 0 || nsteps <= 0) return hipSuccess;
    return streaming ? launch_batch_nt<S, true>(runs_dev, items_dev, nitems, fitems_dev, nfitems, nsteps, ty, parity, first, queues, s)
                     : launch_batch_nt<S, false>(runs_dev, items_dev, nitems, fitems_dev, nfitems, nsteps, ty, parity, first, queues, s);
}

template hipError_t launch_batch<float>(const RunDev<float>*, const Item*, int, const FillItem*,
                                        int, int, int, int, int, int, int*, hipStream_t);
template hipError_t launch_batch<double>(const RunDev<double>*, const Item*, int,
                                         const FillItem*, int, int, int, int, int, int, int*,
                                         hipStream_t);

}  // namespace vlb
