// Device pieces shared by the persistent CG kernels (cg.hip, cg1.hip): the
// coherent loads, the grid barrier, the block to chunk map and the
// deterministic block reductions.
#pragma once
#include "internal.hpp"
#include "stencil.hpp"

#include <hip/hip_runtime.h>

namespace rsr {

__device__ __forceinline__ unsigned long long realtime() { return __builtin_amdgcn_s_memrealtime(); }

// Coherence across XCDs.  Each XCD has its own L2; an agent-scope acquire
// invalidates it.  While the work assignment is unchanged a workgroup owns the
// same tiles in every phase, so its own tile data, the weight planes and the
// local bases stay valid in its L2 and L1.  Only data written by other
// workgroups -- halo cells, reduction partials, deflation coefficients -- is
// read with agent-scope coherent loads (sc1), which do not hit stale lines.
// Writers publish with the release at the barrier arrival.  When the
// assignment changes, one full agent-scope acquire is taken.
__device__ __forceinline__ double cld(const gdbl *p)
{
    typedef __attribute__((address_space(1))) unsigned long long gu64;
    const unsigned long long v = __hip_atomic_load((const gu64 *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}
__device__ __forceinline__ double cld(const double *p) { return cld(gp(p)); }

// Grid barrier, two levels.  Workgroups are split into BAR_GROUPS groups
// (workgroup b in group b % 8, i.e. one group per XCD under round-robin
// dispatch).  Each workgroup publishes its stores with one agent-scope release
// on its group's arrival counter; the last arriver of a group (the counter
// reaching the group's total arrivals up to this barrier) increments the
// global counter and,
// once all groups have arrived, releases its group through the group's epoch
// word.  One contended counter of G arrivals becomes G/8 arrivals per group
// counter plus 8 on the global one, and every group polls its own word.
// All spins use relaxed loads (an acquire inside the loop would invalidate
// the XCD's L2 on every poll); the final acquire is workgroup-scope (see the
// coherence note above).  Every wait is bounded: past the time limit the
// waiting workgroup raises the abort flag and every workgroup leaves the
// kernel at its next barrier, so the grid always drains.
struct BarCtl {
    unsigned long long *glob;   // global counter
    unsigned long long *arr;    // group arrival counter of this workgroup
    unsigned long long *rel;    // group release epoch of this workgroup
    int *abort_flag;
    int ngrp;                   // groups
};

__device__ __forceinline__ BarCtl bar_ctl(const CGArgs &A)
{
    BarCtl b;
    const int ngrp = (A.G % BAR_GROUPS == 0) ? BAR_GROUPS : 1;
    const int grp = blockIdx.x % ngrp;
    char *base = (char *)A.bar;
    b.glob = (unsigned long long *)base;
    b.arr = (unsigned long long *)(base + 256 * (2 + grp));
    b.rel = (unsigned long long *)(base + 256 * (2 + BAR_GROUPS + grp));
    b.abort_flag = A.abort_flag;
    b.ngrp = ngrp;
    return b;
}

__device__ __forceinline__ bool spin_until(unsigned long long *word, unsigned long long target, int *abort_flag,
                                           unsigned long long t0, long long timeout)
{
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if ((long long)(realtime() - t0) > timeout) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// The grid can shrink during the launch (workgroups past the new size leave
// at a loop top), so the arrivals a group counter has seen are tracked in LDS:
// *s_arr is the count before this barrier, and the group's size is the
// current grid size *s_g over the group count.  Only thread 0 touches *s_arr.
template <bool AGENT = false>
__device__ __forceinline__ bool grid_barrier(const BarCtl &b, unsigned long long k, long long timeout, int *s_flag,
                                             unsigned long long *s_arr, const int *s_g)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t0 = realtime();
        bool ok;
        const unsigned long long gsize = (unsigned long long)(*s_g / b.ngrp);
        const unsigned long long old = __hip_atomic_fetch_add(b.arr, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long before = *s_arr;
        *s_arr = before + gsize;
        if (old == before + gsize - 1) {
            // Relaxed: every workgroup of the group wrote its L2 back in the
            // release of its own arrival, which completed before that arrival
            // was counted, so the group's data is in memory before this
            // increment can happen; the same holds for the release word below.
            // (A release here would write the L2 back once more on the
            // barrier's critical path.)
            __hip_atomic_fetch_add(b.glob, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = spin_until(b.glob, k * (unsigned long long)b.ngrp, b.abort_flag, t0, timeout);
            if (ok) __hip_atomic_store(b.rel, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = spin_until(b.rel, k, b.abort_flag, t0, timeout);
        }
        // workgroup scope: other workgroups' data is then read with coherent loads;
        // agent scope: the CU's L1 and the XCD's L2 drop what may be stale, and
        // plain loads see every arrival's stores
        if constexpr (AGENT) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        *s_flag = ok ? 1 : 0;
    }
    __syncthreads();
    return *s_flag != 0;
}

__device__ __forceinline__ int chunk_of_block(int b, int G)
{
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
    // run of chunks so that neighbouring tiles (shared halos) share an L2.
    if (G % 8 == 0) return (b % 8) * (G / 8) + b / 8;
    return b;
}


// Chunk partials are stored value-major: value v of slot k at part[v * ps + k]
// (ps = slots of the launch), so that the reductions, which read one value of
// many consecutive slots per instruction, touch whole cache lines.
//
// Deterministic block-wide sum of cnt (<= NV) consecutive partial values of
// one system: part[(v0 + j) * ps + base + k] over k < nch, in two steps.
// partial_load: each thread accumulates the slots k = threadIdx.x + i * NT in
// registers; block_sum: wave sums, then the waves in order, into out[0..cnt).
template <int NV>
__device__ __forceinline__ void partial_load(const double *part, int ps, int base, int nch, int v0, int cnt,
                                             double (&acc)[NV])
{
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int k = threadIdx.x; k < nch; k += NT) {
        const double *p = part + v0 * ps + base + k;
        // branch-free so that all loads of a slot are in flight together; the
        // clamped index stays inside the used values
        double v[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = cld(p + (j < cnt ? j : cnt - 1) * ps);
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += j < cnt ? v[j] : 0.0;
    }
}

// The wave's sums of cnt (<= NV) per-lane values into wred[0..cnt): up to 16
// values through one transposing reduction (wave_sum16), the rest (and sets of
// at most 4) one by one.
template <int NV>
__device__ __forceinline__ void wave_partials(const double (&v)[NV], int cnt, double *wred)
{
    const int lane = threadIdx.x & 63;
    if constexpr (NV > 4) {
        constexpr int N1 = NV < 16 ? NV : 16;
        double first[N1];
#pragma unroll
        for (int j = 0; j < N1; ++j) first[j] = v[j];
        const double s = wave_sum16<N1>(first);
        if (lane < N1 && lane < cnt) wred[lane] = s;
#pragma unroll
        for (int j = 16; j < NV; ++j)
            if (j < cnt) {
                const double s2 = wave_sum(v[j]);
                if (lane == 0) wred[j] = s2;
            }
    } else {
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < cnt) {
                const double s2 = wave_sum(v[j]);
                if (lane == 0) wred[j] = s2;
            }
    }
}

template <int NV>
__device__ void block_sum(const double (&acc)[NV], int cnt, double *out, double *red)
{
    const int wid = threadIdx.x >> 6;
    wave_partials<NV>(acc, cnt, red + wid * NVP);
    __syncthreads();
    if (threadIdx.x < cnt) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * NVP + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int NV>
__device__ void block_reduce_partials(const double *part, int ps, int base, int nch, int v0, int cnt, double *out,
                                      double *red)
{
    double acc[NV];
    partial_load<NV>(part, ps, base, nch, v0, cnt, acc);
    block_sum<NV>(acc, cnt, out, red);
}

// Adds the block-wide sums of cnt per-thread values (fixed order) to acc[0..cnt).
template <int NV>
__device__ __forceinline__ void block_accumulate(const double (&v)[NV], int cnt, double *acc, double *red)
{
    const int wid = threadIdx.x >> 6;
    wave_partials<NV>(v, cnt, red + wid * NVP);
    __syncthreads();
    if (threadIdx.x < cnt) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * NVP + threadIdx.x];
        acc[threadIdx.x] += s;
    }
    __syncthreads();
}

constexpr int NBW = 6;    // window rows per thread whose loads are issued together (three fields each)
constexpr int NBW2 = 18;  // the same for the two-pass stencil phase (ph alone): a 72-row window in one round
constexpr int NBE = 2;   // interior pixels per thread whose local-basis loads are issued together

}  // namespace rsr
