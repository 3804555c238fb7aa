// Device work queues for the stages whose boxes depend on other boxes of the
// same stage (the upward pass: a parent needs its children's proxy charges;
// the local values: a box needs its anchor ancestor's polynomial).
//
// One launch covers every level.  The items (box indices) sit in a list in
// dependency order (finest level first for the upward pass, coarsest first
// for the local values); the workgroups of a persistent grid take them one
// at a time from an atomic head.  Before computing an item a workgroup waits
// until the items it depends on have published their output (a per-item
// flag), and after computing it publishes its own.
//
// Why every wait ends: a workgroup takes an item only while it is resident,
// and an item's dependencies come earlier in the list, so each of them is
// held by a resident workgroup (or done) when the item is taken; by
// induction over the list every item completes.  The wait is bounded all the
// same (q.tmax wall-clock ticks): a wait that runs out counts itself in
// `fail` and goes on, so the kernel always exits; the plan reports the count.
//
// Visibility across the eight XCDs (each with its own L2, not coherent with
// the others for ordinary accesses): whatever one item writes and another
// item of the same launch reads (proxy charges, local values) is stored and
// loaded with relaxed agent-scope atomics, which go past the non-coherent
// caches; a producer's threads wait until their stores have completed before
// the workgroup barrier after which one thread sets the flag.  No
// agent-scope fence is used: on this chip such a fence writes back or
// invalidates a whole L2.  Everything else an item reads was written by
// earlier launches.
//
// The loop's control is kept uniform (the item index goes through a scalar
// register), so that the compiler keeps it a single loop with the
// single-thread hand-out inside it; with a per-lane index it split the loop
// so that the other lanes went on past the barrier with the old item.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dmk_internal.h"

namespace dmk {

struct WorkQ {
    int32_t *head;        // next item to hand out (zeroed before the launch)
    int32_t *done;        // per-slot flags: 1 once that item's output is published
    const int32_t *list;  // items in dependency order
    const int32_t *slot;  // box -> flag index
    int32_t *fail;        // waits that ran out of time (sticky, plan-owned)
    int32_t n;            // items
    int64_t tmax;         // longest wait, in wall-clock ticks
};

// loads and stores of the data passed between items of one launch (COH), or
// ordinary ones
template <bool COH, typename T>
__device__ __forceinline__ T ld_c(const T *p)
{
    if constexpr (COH)
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}
template <bool COH, typename T>
__device__ __forceinline__ void st_c(T *p, T v)
{
    if constexpr (COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// copy n values to LDS with the workgroup's NT threads; COH: the coherent
// loads go out in batches of 8 before their values are used (each atomic
// load followed by its own wait would cost a memory round trip per value)
template <bool COH, int NT, typename T>
__device__ __forceinline__ void copy_to_lds(T *dst, const T *src, int n)
{
    if constexpr (!COH) {
        for (int t = threadIdx.x; t < n; t += NT) dst[t] = src[t];
    } else {
        for (int t0 = threadIdx.x; t0 < n; t0 += 8 * NT) {
            T r[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u * NT;
                r[u] = t < n ? ld_c<true>(src + t) : T(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u * NT;
                if (t < n) dst[t] = r[u];
            }
        }
    }
}

// wait (one thread) until the item of box b has published its output, at most
// q.tmax ticks of the constant-rate wall clock
__device__ __forceinline__ void wait_done(const WorkQ &q, int32_t b)
{
    const int32_t *f = q.done + q.slot[b];
    if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const int64_t t0 = (int64_t)wall_clock64();
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        if ((int64_t)wall_clock64() - t0 > q.tmax) {
            atomicAdd(q.fail, 1);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// this thread's memory operations so far have completed (vmcnt 0; the
// workgroup fence keeps the compiler from moving them past the wait)
__device__ __forceinline__ void complete_stores()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xf << 8));
}

// the persistent loop of a queue-fed kernel: `wait(b)` is called by every
// thread (it waits on the dependencies of box b from some threads), `body(b)`
// computes box b with the whole workgroup, loading its dependencies and
// storing its output with ld_c/st_c<true>
template <class Wait, class Body>
__device__ __forceinline__ void queue_loop(const WorkQ &q, Wait wait, Body body)
{
    __shared__ int32_t s_item;
    if (threadIdx.x == 0) s_item = atomicAdd(q.head, 1);
    __syncthreads();
    int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    while (it < q.n) {
        const int32_t b = __builtin_amdgcn_readfirstlane(q.list[it]);
        wait(b);
        __syncthreads();
        body(b);
        complete_stores();
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(q.done + q.slot[b], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_item = atomicAdd(q.head, 1);
        }
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(s_item);
    }
}

// one item per workgroup (the grid has one workgroup per item): the same
// protocol without the loop, for bodies whose registers do not survive one
template <class Wait, class Body>
__device__ __forceinline__ void queue_item(const WorkQ &q, Wait wait, Body body)
{
    __shared__ int32_t s_item;
    if (threadIdx.x == 0) s_item = atomicAdd(q.head, 1);
    __syncthreads();
    const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= q.n) return;
    const int32_t b = __builtin_amdgcn_readfirstlane(q.list[it]);
    wait(b);
    __syncthreads();
    body(b);
    complete_stores();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(q.done + q.slot[b], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- host
// workgroups of a kernel that fit on the device at once (the persistent grid
// of a queue-fed kernel; more would only wait for a slot)
template <typename K>
inline unsigned resident_blocks(K kernel, int nthreads, size_t lds)
{
    int dev = 0, ncu = 0, per = 0;
    DMK_HIP(hipGetDevice(&dev));
    DMK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    DMK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, nthreads, lds));
    return (unsigned)std::max(1, per) * (unsigned)std::max(1, ncu);
}

// the longest wait of a queue-fed kernel, in ticks of the device's
// constant-rate wall clock: 200 ms, far beyond any real wait (a whole stage
// takes a few ms), so that a wait that runs out means a fault
inline int64_t queue_wait_ticks()
{
    static const int64_t ticks = [] {
        int dev = 0, khz = 0;
        DMK_HIP(hipGetDevice(&dev));
        DMK_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        return (int64_t)std::max(khz, 1000) * 200;
    }();
    return ticks;
}

namespace {
// clears the heads and flags of the queues (a kernel, so that it can sit in a
// captured graph)
__global__ void __launch_bounds__(256) k_queue_reset(int32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) p[i] = 0;
}
}  // namespace

// clears n control words (head and flags) of a queue
static inline void reset_queue(int32_t *p, int64_t n, hipStream_t s)
{
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_queue_reset, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(256), 0, s, p, n);
}

// the queues' control words (workspace, 8 + nfout + nanc ints): [0, 4 + nfout)
// the upward pass's head and flags, [4 + nfout, 8 + nfout + nanc) the local
// values' (cleared by the stage's reset kernel before each of its launches)
inline WorkQ upward_queue(Plan *Pl)
{
    return WorkQ{Pl->qctl, Pl->qctl + 4, Pl->l_fout_up, Pl->proxy_slot, Pl->q_fail, (int32_t)Pl->nfout,
                 queue_wait_ticks()};
}
inline WorkQ local_queue(Plan *Pl)
{
    int32_t *base = Pl->qctl + 4 + Pl->nfout;
    return WorkQ{base, base + 4, Pl->l_anc, Pl->local_slot, Pl->q_fail, (int32_t)Pl->nanc, queue_wait_ticks()};
}
inline int64_t queue_ctl_words(const Plan *Pl) { return 8 + Pl->nfout + Pl->nanc; }


}  // namespace dmk
