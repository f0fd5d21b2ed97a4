// oci_device.hpp -- device helpers shared by the gfx950 iteration kernels of
// liboci: step statuses, fixed-order reductions and the grid barrier fused
// with the reduction of per-workgroup sums.  Not part of the public ABI.
#pragma once

#include "oci_internal.hpp"

namespace oci {

constexpr int OK = 0, NOT_CONVERGED = 1, NONFINITE = 2;

// The stopping rule after `iters` iterations (1, 2, ...) from the norm e of
// the last change and e_prev of the one before (NaN for the first): a
// non-finite e ends the step; a fixed count ends it after that many; else
// e < tol (1 - e / e_prev) from the second iteration on (e = 0 included);
// else the iteration cap.  Returns 1 when the step ends, with its status.
__device__ inline int stop_rule(const Slab &S, int iters, double e, double e_prev, int *status) {
    *status = OK;
    if (!isfinite(e)) {
        *status = NONFINITE;
        return 1;
    }
    if (S.fixed_iters > 0) return iters >= S.fixed_iters;
    if (iters >= 2 && (e == 0.0 || e < S.tol * (1.0 - e / e_prev))) return 1;
    if (iters >= S.max_iters) {
        *status = NOT_CONVERGED;
        return 1;
    }
    return 0;
}

// --------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-shape workgroup sum (same pairing every call, so deterministic).
__device__ inline double block_sum(double v, double *s_tmp) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_tmp[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) t += s_tmp[w];
    __syncthreads();
    return t;  // valid in thread 0
}

template <int BS>
__device__ inline double block_sum_t(double v, double *s_tmp) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BS / 64; ++w) t += s_tmp[w];
    __syncthreads();
    return t;  // valid in thread 0
}

// Grid barrier over the co-resident workgroups of one launch, once per
// iteration l, fused with the reduction of the per-workgroup sums.
// Counters only grow during a step (they are reset before it), so barrier l
// has a known target and nobody reads shared state to learn it: workgroups
// arrive at their group's counter, the last of a group arrives at the top
// counter, and everybody waits for the top counter to reach (l + 1) x groups.
// Arrivals are agent-scope acquire-release read-modify-writes (publishing the
// workgroup's stores, its partial sum included); the wait uses relaxed loads
// and one agent-scope acquire at the end, so no cache maintenance happens
// inside the spin.  Then every workgroup sums the partials of iteration l in
// the same fixed order, so all of them hold the identical total and take the
// identical stopping decision with no second round trip.  The spin is
// bounded: on expiry the control block's err flag is raised and the caller
// leaves its loop, so the grid always drains.
constexpr long kSpinLimit = 1L << 25;

template <int BS>
__device__ inline bool grid_sync_sum(const Slab &S, unsigned wg, unsigned nwg, int l, double wg_sum, int *s_flag,
                                     double *s_tmp, double *total) {
    double *part = S.partials + (size_t)(l & 1) * nwg;
    if (threadIdx.x == 0) part[wg] = wg_sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gsz_all = (unsigned)S.bar_gsz;
        const unsigned grp = wg / gsz_all;
        const unsigned ngrp = (nwg + gsz_all - 1) / gsz_all;
        const unsigned gsz = (grp + 1 == ngrp) ? nwg - grp * gsz_all : gsz_all;
        const uint64_t round = (uint64_t)l + 1;
        uint64_t *gc = S.bar + (size_t)(2 + grp) * kBarStride;
        const uint64_t og = __hip_atomic_fetch_add(gc, (uint64_t)1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (og + 1 == round * gsz)
            (void)__hip_atomic_fetch_add(S.bar, (uint64_t)1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int bad = 0;
        long spins = 0;
        while (__hip_atomic_load(S.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < round * ngrp) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                __hip_atomic_store(&S.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bad = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_flag[2] = bad;
    }
    __syncthreads();
    double v = 0.0;
    for (unsigned k = threadIdx.x; k < nwg; k += BS) v += part[k];
    v = block_sum_t<BS>(v, s_tmp);
    if (threadIdx.x == 0) s_tmp[BS / 64] = v;
    __syncthreads();
    *total = s_tmp[BS / 64];
    return s_flag[2] == 0;
}

// Agent-coherent accesses: relaxed agent-scope atomics, which gfx950 performs
// at the device's coherence point (the loads and stores carry sc1) with no
// L2 writeback or invalidate.  Data that one workgroup writes and another
// reads inside a launch goes through these.
__device__ inline double ld_coherent(const double *p) {
    return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<double *>(p)),
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline void st_coherent(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this thread's memory operations have completed (vmcnt = 0;
// expcnt and lgkmcnt left alone).
__device__ inline void wait_memory() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Grid barrier and reduction without cache maintenance, for launches whose
// cross-workgroup data all goes through ld_coherent / st_coherent: every
// thread waits for its own stores to complete, the workgroup meets, thread 0
// publishes the workgroup's partial and arrives with relaxed atomics (the
// release of the memory model minus the L2 writeback, which only non-coherent
// data would need).  The workgroup whose arrival completes the count raises
// the release word at once; the others wait for it (the acquire minus the L2
// invalidate, so the workgroups keep their cached read-only data).  Then every
// workgroup sums the published partials itself, in ascending workgroup order
// through the same fixed-shape reduction, so all hold the same total without
// a round trip through a published total.  Round `round` (0, 1, ...) must grow
// by one per call; the partials alternate between two rows (a row is
// rewritten two rounds later, after every workgroup has read it).  Every wait
// is bounded as in grid_sync_sum.
template <int BS>
__device__ inline bool grid_sync_coherent(const Slab &S, unsigned wg, unsigned nwg, int round, double wg_sum,
                                          int *s_flag, double *s_tmp, double *total) {
    double *part = S.partials + (size_t)(round & 1) * nwg;
    uint64_t *release = S.bar + kBarStride;
    const uint64_t target = (uint64_t)round + 1;
    wait_memory();
    __syncthreads();
    if (threadIdx.x == 0) {
        st_coherent(part + wg, wg_sum);
        wait_memory();
        const unsigned gsz_all = (unsigned)S.bar_gsz;
        const unsigned grp = wg / gsz_all;
        const unsigned ngrp = (nwg + gsz_all - 1) / gsz_all;
        const unsigned gsz = (grp + 1 == ngrp) ? nwg - grp * gsz_all : gsz_all;
        uint64_t *gc = S.bar + (size_t)(2 + grp) * kBarStride;
        int last = 0;
        const uint64_t og = __hip_atomic_fetch_add(gc, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (og + 1 == target * gsz) {
            const uint64_t ot = __hip_atomic_fetch_add(S.bar, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = ot + 1 == target * ngrp;
        }
        int bad = 0;
        if (last) {
            __hip_atomic_store(release, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(&S.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bad = 1;
                    break;
                }
            }
        }
        s_flag[2] = bad;
    }
    __syncthreads();
    const int bad = s_flag[2];
    double v = 0.0;
    if (!bad)
        for (unsigned k = threadIdx.x; k < nwg; k += BS) v += ld_coherent(part + k);
    v = block_sum_t<BS>(v, s_tmp);
    if (threadIdx.x == 0) s_tmp[BS / 64] = bad ? __builtin_nan("") : v;
    __syncthreads();
    *total = s_tmp[BS / 64];
    return bad == 0;
}

// Orders the LDS accesses of one wave before and after it (the wave's LDS
// operations complete in issue order; this only keeps the compiler from
// moving them across).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace oci
