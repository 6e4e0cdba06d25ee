// bdis_persist.hpp -- one persistent launch for a whole batch of stereo pairs.
//
// The host flattens every block of every kernel of the path (pyramid levels,
// then per level from the coarsest down: LK + posterior blocks, then
// densification blocks) for all pairs into one task list in dependency
// order.  Workgroup g runs tasks g, g + G, g + 2G, ... in order.  Before a
// task runs, the workgroup waits until the jobs it reads from are complete
// (per-job completion counters); after it, it bumps its own job's counter.
// A task only ever waits on tasks earlier in the list, and the grid is sized
// so that every workgroup is resident, so the earliest unfinished task can
// always run: the launch drains.  Waits are bounded: a wait that exceeds the
// spin limit sets the error flag and the task proceeds (results are then
// wrong, the host reports the error), so no wave can spin forever.
#pragma once
#include "bdis_kernels.hpp"

namespace bdis {

enum { PK_PYR = 0, PK_LK = 1, PK_DENSE = 2 };

struct PJob {
    int *done;       // this job's completion counter (blocks finished)
    const int *dep0; // jobs this one reads: counter and the count meaning done
    const int *dep1;
    int kind;        // PK_*
    int patch;       // LK patch side
    int u8;          // level-0 images (uint8) or a pyramid level
    int kp;          // index of the job's KParams
    int need0;
    int need1;
    PyrJob pyr;
    LkJob lk;
    DenseJob dense;
};
static_assert(sizeof(PJob) == 3 * 8 + 6 * 4 + sizeof(PyrJob) + sizeof(LkJob) + sizeof(DenseJob),
              "PJob must have no padding");

struct PTask {
    int job;
    int lb;  // block index inside the job
};

__device__ __forceinline__ void wait_count(const int *c, int need, int *err, int limit) {
    if (!c) return;
    int spins = 0;
    while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > limit) {
            __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
}

// Clears the completion counters and the error flag of a persistent run
// (a kernel, not a memset, so the pair can sit in a replayed graph).
__global__ __launch_bounds__(kBlock) void k_reset(int *counters, int n) {
    for (int i = (int)(blockIdx.x * kBlock + threadIdx.x); i < n; i += (int)(gridDim.x * kBlock))
        counters[i] = 0;
}

template <typename T, int P, int WN>
__device__ __forceinline__ void lk_task(const PJob &J, int lb, const KParams &kp, T *Rs) {
    if (J.u8) lk_block<T, P, true, WN>(J.lk, lb, kp, Rs);
    else lk_block<T, P, false, WN>(J.lk, lb, kp, Rs);
}

// Patch sides the persistent kernel is built for (the autotuner's space).
__host__ __device__ constexpr bool persist_patch_ok(int p) { return p == 8 || p == 12; }

// WN: the window bound of the LK tasks, as for k_lk (the same code, so the
// results equal those of the launch-per-level executions bit for bit).
template <typename T, int WN>
__global__ __launch_bounds__(kBlock) void k_persist(const PTask *__restrict__ tasks, int ntasks,
                                                    const PJob *__restrict__ jobs,
                                                    const KParams *__restrict__ kps, int *err,
                                                    int spin_limit) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *Rs = reinterpret_cast<T *>(smem);
    // the last dependency this workgroup saw satisfied: consecutive tasks of
    // one job skip the wait
    const int *seen0 = nullptr, *seen1 = nullptr;
    int seen_need0 = 0, seen_need1 = 0;
    for (int t = (int)blockIdx.x; t < ntasks; t += (int)gridDim.x) {
        const PTask tk = tasks[t];
        const PJob &J = jobs[tk.job];
        const bool fresh = J.dep0 != seen0 || J.need0 != seen_need0 || J.dep1 != seen1 ||
                           J.need1 != seen_need1;
        if (fresh) {
            if (threadIdx.x == 0) {
                wait_count(J.dep0, J.need0, err, spin_limit);
                wait_count(J.dep1, J.need1, err, spin_limit);
            }
            seen0 = J.dep0; seen_need0 = J.need0;
            seen1 = J.dep1; seen_need1 = J.need1;
        }
        __syncthreads();
        const KParams &kp = kps[J.kp];
        switch (J.kind) {
        case PK_PYR:
            if (J.u8) pyr_block<T, true>(J.pyr, tk.lb, kp);
            else pyr_block<T, false>(J.pyr, tk.lb, kp);
            break;
        case PK_LK:
            if (J.patch == 8) lk_task<T, 8, WN>(J, tk.lb, kp, Rs);
            else lk_task<T, 12, WN>(J, tk.lb, kp, Rs);
            break;
        default:
            if (J.u8) dense_block<T, true>(J.dense, tk.lb, kp);
            else dense_block<T, false>(J.dense, tk.lb, kp);
            break;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_fetch_add(J.done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace bdis
