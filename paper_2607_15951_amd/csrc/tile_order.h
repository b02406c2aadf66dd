// tile_order.h -- the blend's heaviest-first dispatch order: a counting sort
// of the tiles by descending cost bucket, run by one workgroup.  Shared by
// the order kernel (blend.hip: the first frame of a layout, ordered by list
// length) and the projection launch (project.hip: later frames, ordered by
// the previous frame's walked entries, in one extra workgroup that runs
// beside the projection instead of on the frame's critical path).
#pragma once

#include "gs_internal.h"

namespace gsmi {

// Log-scale bucket of a tile's cost: exact below 128, then 32 buckets per
// octave (costs within about 3% share one); 0 .. 927.
constexpr int kOrderBuckets = 1024;
__device__ __forceinline__ int cost_bucket(uint32_t c)
{
    if (c < 128u) return (int)c;
    const int e = 31 - __clz(c);   // 7 .. 31
    return 128 + (e - 7) * 32 + (int)((c >> (e - 5)) & 31u);
}

__device__ __forceinline__ uint32_t tile_cost_of(const uint32_t* cost, const uint32_t* offsets, int64_t t)
{
    return cost ? cost[t] : offsets[t + 1] - offsets[t];
}

// Writes order[0 .. tiles): all tiles, heaviest cost bucket first, by cost[t]
// or (cost null) by list length.  Called by every thread of a workgroup of
// kThreads; LDS: hist[kOrderBuckets], wsum[kThreads / 64] and, optionally,
// kept[kept_n] (each kept tile's bucket between the passes; tiles past
// kept_n load their cost again).  The first pass loads kOrderPre costs per
// thread before using any (a load under its own branch is waited for before
// the next one issues) and counts the buckets with LDS atomics; the second
// claims each tile's slot with one more atomic.  Within a bucket the order is
// whatever the atomics give: the order only decides when each tile's
// workgroup starts, never what it computes.  (Plain atomics, colliding where
// many tiles share a bucket, cost less issue than grouping the lanes of a
// bucket with ballots.)
constexpr int kOrderPre = 8;
template <int kThreads>
__device__ __forceinline__ void order_heaviest_first(const uint32_t* __restrict__ cost,
                                                     const uint32_t* __restrict__ offsets, int64_t tiles,
                                                     uint32_t* __restrict__ order, uint32_t* hist, uint32_t* wsum,
                                                     uint16_t* kept, int64_t kept_n)
{
    static_assert(kOrderBuckets % kThreads == 0, "whole buckets per thread in the scan");
    constexpr int kPer = kOrderBuckets / kThreads;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < kOrderBuckets; i += kThreads) hist[i] = 0u;
    __syncthreads();
    constexpr int64_t kStep = (int64_t)kThreads * kOrderPre;
    for (int64_t t0 = 0; t0 < tiles; t0 += kStep) {
        uint32_t c[kOrderPre];
#pragma unroll
        for (int k = 0; k < kOrderPre; ++k) {
            const int64_t t = t0 + k * kThreads + tid;
            c[k] = tile_cost_of(cost, offsets, t < tiles ? t : 0);
        }
#pragma unroll
        for (int k = 0; k < kOrderPre; ++k) {
            const int64_t t = t0 + k * kThreads + tid;
            if (t < tiles) {
                const int b = cost_bucket(c[k]);
                atomicAdd(&hist[b], 1u);
                if (t < kept_n) kept[t] = (uint16_t)b;
            }
        }
    }
    __syncthreads();
    // start of each bucket in descending bucket order: thread tid holds
    // positions tid * kPer .. + kPer - 1 of that order (bucket 1023 - f at
    // position f), scanned exclusively across the workgroup
    uint32_t own[kPer], run = 0u;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        own[k] = hist[kOrderBuckets - 1 - (tid * kPer + k)];
        run += own[k];
    }
    uint32_t x = run;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t acc = x - run;
    for (int w = 0; w < wave; ++w) acc += wsum[w];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        hist[kOrderBuckets - 1 - (tid * kPer + k)] = acc;   // now the bucket's next free slot
        acc += own[k];
    }
    __syncthreads();
    for (int64_t t0 = 0; t0 < tiles; t0 += kStep) {
        uint32_t c[kOrderPre];
        const bool reload = t0 + kStep > kept_n;   // uniform: whole steps past the kept tiles
        if (reload) {
#pragma unroll
            for (int k = 0; k < kOrderPre; ++k) {
                const int64_t t = t0 + k * kThreads + tid;
                c[k] = tile_cost_of(cost, offsets, t < tiles ? t : 0);
            }
        }
#pragma unroll
        for (int k = 0; k < kOrderPre; ++k) {
            const int64_t t = t0 + k * kThreads + tid;
            if (t < tiles) {
                const int b = reload ? cost_bucket(c[k]) : (int)kept[t];
                order[atomicAdd(&hist[b], 1u)] = (uint32_t)t;
            }
        }
    }
}

}  // namespace gsmi
