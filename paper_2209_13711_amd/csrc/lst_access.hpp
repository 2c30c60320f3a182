// Device-side accessors of the arena shared by the kernel files: the
// overflow flag and the compact index over stored quintuplets.
#pragma once

#include "lst_internal.hpp"

namespace lst {

__device__ __forceinline__ bool upstream_overflow(const EvDev &E)
{
    return E.gc[GC_OVERFLOW] != 0u;
}

// per-event index of grouped hit h (either storage)
__device__ __forceinline__ int32_t hit_orig(const EvDev &E, int32_t h)
{
    return E.half16 ? (int32_t)E.hsort_h[h].y : __float_as_int(E.hsort[h].w);
}

__device__ __forceinline__ int32_t t5_md(const EvDev &E, int32_t t, int j)
{
    switch (j) {
    case 0: return E.t5_md0[t];
    case 1: return E.t5_md1[t];
    case 2: return E.t5_md2[t];
    case 3: return E.t5_md3[t];
    default: return E.t5_md4[t];
    }
}

__device__ __forceinline__ int32_t t5_hit(const EvDev &E, int32_t t, int j)
{
    const int32_t md = t5_md(E, t, j >> 1);
    return (j & 1) ? E.md_hup[md] : E.md_hlo[md];
}

// Compact index over the stored objects of one type: the block keeps the
// prefix of the NSH region sizes in LDS; a thread maps v to its array index
// with a binary search over it.
__device__ __forceinline__ uint32_t obj_prefix(const EvDev &E, int type, uint32_t *s_pre)
{
    if (threadIdx.x == 0) {
        const uint32_t rc = E.rc[type];
        uint32_t acc = 0;
        for (int r = 0; r < NSH; ++r) {
            s_pre[r] = acc;
            const uint32_t c = E.gc[gc_shard(type, r)];
            acc += c < rc ? c : rc;
        }
        s_pre[NSH] = acc;
    }
    __syncthreads();
    return s_pre[NSH];
}

__device__ __forceinline__ int32_t obj_at(const EvDev &E, int type, const uint32_t *s_pre, uint32_t v)
{
    int lo = 0, hi = NSH - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return (int32_t)((uint32_t)lo * E.rc[type] + (v - s_pre[lo]));
}

__device__ __forceinline__ uint32_t t5_prefix(const EvDev &E, uint32_t *s_pre)
{
    return obj_prefix(E, OT_T5, s_pre);
}

__device__ __forceinline__ int32_t t5_at(const EvDev &E, const uint32_t *s_pre, uint32_t v)
{
    return obj_at(E, OT_T5, s_pre, v);
}

}  // namespace lst
