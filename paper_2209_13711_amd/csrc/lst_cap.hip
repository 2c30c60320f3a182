// Per-module capacities of the object arrays.
//
// The paper stores every object kind in arrays of a fixed capacity per
// module and sets that capacity at a high quantile (99.9 % or 99.99 %) of the
// per-module occupancy, which shrinks the memory footprint about fivefold for
// a loss of 1-2 % in efficiency (Sec. 3); a module holding more objects than
// its capacity loses the rest.  This library keeps its compact layout and
// reproduces the selection: after a stage, each module (slot) holding more
// than `cap` objects of the stage's kind keeps the `cap` whose tuples of
// per-event hit indices are smallest (lexicographically), the module of an
// object being that of its first mini-doublet.  The rule is fixed so that
// the oracle can reproduce it; which objects the paper's GPU loses depends on
// thread timing.  Later stages see only the kept objects.
//
// Three passes per kind, all only in this mode:
//   rank    one wave per slot: a slot above its capacity ranks its objects
//           (grouped by first MD, each MD's objects consecutive) and flags
//           those ranked cap or later;
//   compact one block per shard region: a stable in-place compaction of the
//           kind's arrays, recording for every position the number of kept
//           objects before it in its shard;
//   fix     per slot (MDs) or per MD (the others): the group ranges mapped
//           through those prefixes.
#include "lst_access.hpp"

namespace lst {

__device__ __forceinline__ int cap_lane() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t cap_wave_sum(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// an MD's (lower, upper) per-event hit indices as one lexicographic key
__device__ __forceinline__ uint64_t md_key(const EvDev &E, int32_t m)
{
    const uint32_t lo = (uint32_t)hit_orig(E, E.md_hlo[m]);
    const uint32_t up = (uint32_t)hit_orig(E, E.md_hup[m]);
    return ((uint64_t)lo << 32) | up;
}

// Per kind: the range of the objects of an MD, and the keys of an object's
// MDs after the first (all objects of one range share the first).
template <int KIND> struct CapOf;

template <> struct CapOf<OT_SEG> {
    static constexpr int NT = 1;
    __device__ static int32_t start(const EvDev &E, int32_t m) { return E.seg_start[m]; }
    __device__ static int32_t cnt(const EvDev &E, int32_t m) { return E.seg_cnt[m]; }
    __device__ static void tail(const EvDev &E, int32_t o, uint64_t *k) { k[0] = md_key(E, E.seg_out[o]); }
};

template <> struct CapOf<OT_T3> {
    static constexpr int NT = 2;
    __device__ static int32_t start(const EvDev &E, int32_t m) { return E.t3_start[m]; }
    __device__ static int32_t cnt(const EvDev &E, int32_t m) { return E.t3_cnt[m]; }
    __device__ static void tail(const EvDev &E, int32_t o, uint64_t *k)
    {
        k[0] = md_key(E, E.t3_b[o]);
        k[1] = md_key(E, E.t3_c[o]);
    }
};

template <> struct CapOf<OT_T5> {
    static constexpr int NT = 4;
    __device__ static int32_t start(const EvDev &E, int32_t m) { return E.t5_start[m]; }
    __device__ static int32_t cnt(const EvDev &E, int32_t m) { return E.t5_cnt[m]; }
    __device__ static void tail(const EvDev &E, int32_t o, uint64_t *k)
    {
        k[0] = md_key(E, E.t5_md1[o]);
        k[1] = md_key(E, E.t5_md2[o]);
        k[2] = md_key(E, E.t5_md3[o]);
        k[3] = md_key(E, E.t5_md4[o]);
    }
};

template <int N>
__device__ __forceinline__ bool keys_less(const uint64_t *a, const uint64_t *b)
{
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (a[i] != b[i]) return a[i] < b[i];
    return false;
}

__device__ __forceinline__ void count_drops(const EvDev &E, int type, int slot, uint32_t dropped)
{
    dropped = cap_wave_sum(dropped);
    if (cap_lane() == 0 && dropped) {
        const int n_mod = E.cap_slots / E.cap_ev;
        atomicAdd(&E.gc[GC_DROP + type], dropped);
        atomicAdd(&E.cap_nd[(slot / n_mod) * OT_COUNT + type], dropped);
    }
}

// ---------------------------------------------------------------- rank
// MDs: the MDs of a slot are its objects; rank = MDs of the slot with a
// smaller key.
__global__ __launch_bounds__(BLOCK) void k_cap_rank_md(EvDev E, int32_t cap)
{
    if (upstream_overflow(E)) return;
    const int n_slots = E.desc[D_NSLOTS];
    const int l = cap_lane();
    const int nw = gridDim.x * WAVES;
    for (int slot = blockIdx.x * WAVES + (int)(threadIdx.x >> 6); slot < n_slots; slot += nw) {
        const int32_t mc = E.md_cnt[slot];
        if (mc <= cap) continue;
        const int32_t ms = E.md_start[slot];
        uint32_t dropped = 0;
        for (int32_t i = l; i < mc; i += 64) {
            const uint64_t k = md_key(E, ms + i);
            int32_t rank = 0;
            for (int32_t j = 0; j < mc; ++j) rank += md_key(E, ms + j) < k;
            if (rank >= cap) {
                E.cap_drop[ms + i] = 1;
                ++dropped;
            }
        }
        count_drops(E, OT_MD, slot, dropped);
    }
}

// Segments, triplets, quintuplets: the objects of a slot are those of its
// MDs.  rank(o) = objects of the slot's MDs with a smaller first-MD key,
// plus the objects of o's own MD with a smaller tail.
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_cap_rank(EvDev E, int32_t cap)
{
    using C = CapOf<KIND>;
    if (upstream_overflow(E)) return;
    const int n_slots = E.desc[D_NSLOTS];
    const int l = cap_lane();
    const int nw = gridDim.x * WAVES;
    for (int slot = blockIdx.x * WAVES + (int)(threadIdx.x >> 6); slot < n_slots; slot += nw) {
        const int32_t mc = E.md_cnt[slot];
        if (mc <= 0) continue;
        const int32_t ms = E.md_start[slot];
        uint32_t part = 0;
        for (int32_t i = l; i < mc; i += 64) part += (uint32_t)C::cnt(E, ms + i);
        if (cap_wave_sum(part) <= (uint32_t)cap) continue;
        uint32_t dropped = 0;
        for (int32_t i = 0; i < mc; ++i) {      // the same MD in every lane
            const int32_t m = ms + i;
            const uint64_t km = md_key(E, m);
            uint32_t below = 0;
            for (int32_t j = l; j < mc; j += 64)
                if (md_key(E, ms + j) < km) below += (uint32_t)C::cnt(E, ms + j);
            const uint32_t base = cap_wave_sum(below);
            const int32_t st = C::start(E, m), c = C::cnt(E, m);
            for (int32_t o = l; o < c; o += 64) {
                uint64_t ko[C::NT];
                C::tail(E, st + o, ko);
                uint32_t within = 0;
                for (int32_t q = 0; q < c; ++q) {
                    uint64_t kq[C::NT];
                    C::tail(E, st + q, kq);
                    within += keys_less<C::NT>(kq, ko);
                }
                if (base + within >= (uint32_t)cap) {
                    E.cap_drop[st + o] = 1;
                    ++dropped;
                }
            }
        }
        count_drops(E, KIND, slot, dropped);
    }
}

// ---------------------------------------------------------------- compact
// The fields of one object of each kind, moved together.
struct MdRec {
    int32_t hlo, hup, slot;
    int4 nbr;
    float4 p0, p1, p2;
    float bend, atol;
    uint8_t bar;
};
__device__ __forceinline__ MdRec rec_load(const EvDev &E, int32_t i, MdRec *)
{
    MdRec r;
    r.hlo = E.md_hlo[i]; r.hup = E.md_hup[i]; r.slot = E.md_slot[i]; r.nbr = E.md_nbr[i];
    r.p0 = E.md_p0[i]; r.p1 = E.md_p1[i]; r.p2 = E.md_p2[i];
    r.bend = E.md_bend[i]; r.atol = E.md_atol[i]; r.bar = E.md_bar[i];
    return r;
}
__device__ __forceinline__ void rec_store(const EvDev &E, int32_t i, const MdRec &r)
{
    E.md_hlo[i] = r.hlo; E.md_hup[i] = r.hup; E.md_slot[i] = r.slot; E.md_nbr[i] = r.nbr;
    E.md_p0[i] = r.p0; E.md_p1[i] = r.p1; E.md_p2[i] = r.p2;
    E.md_bend[i] = r.bend; E.md_atol[i] = r.atol; E.md_bar[i] = r.bar;
}

struct SegRec { int32_t in, out; };
__device__ __forceinline__ SegRec rec_load(const EvDev &E, int32_t i, SegRec *)
{
    return SegRec{E.seg_in[i], E.seg_out[i]};
}
__device__ __forceinline__ void rec_store(const EvDev &E, int32_t i, const SegRec &r)
{
    E.seg_in[i] = r.in; E.seg_out[i] = r.out;
}

struct T3Rec { int32_t a, b, c; float k; };
__device__ __forceinline__ T3Rec rec_load(const EvDev &E, int32_t i, T3Rec *)
{
    return T3Rec{E.t3_a[i], E.t3_b[i], E.t3_c[i], E.t3_k[i]};
}
__device__ __forceinline__ void rec_store(const EvDev &E, int32_t i, const T3Rec &r)
{
    E.t3_a[i] = r.a; E.t3_b[i] = r.b; E.t3_c[i] = r.c; E.t3_k[i] = r.k;
    E.t3_veto[i] = 0;
}

struct T5Rec { int32_t m[5]; float score; };
__device__ __forceinline__ T5Rec rec_load(const EvDev &E, int32_t i, T5Rec *)
{
    T5Rec r;
    r.m[0] = E.t5_md0[i]; r.m[1] = E.t5_md1[i]; r.m[2] = E.t5_md2[i];
    r.m[3] = E.t5_md3[i]; r.m[4] = E.t5_md4[i];
    r.score = E.t5_score[i];
    return r;
}
__device__ __forceinline__ void rec_store(const EvDev &E, int32_t i, const T5Rec &r)
{
    E.t5_md0[i] = r.m[0]; E.t5_md1[i] = r.m[1]; E.t5_md2[i] = r.m[2];
    E.t5_md3[i] = r.m[3]; E.t5_md4[i] = r.m[4];
    E.t5_score[i] = r.score;
    E.t5_keep[i] = 0;
    E.t5_veto[i] = 0;
}

// One block per shard region: kept objects move down, in order.  Every
// thread loads its object before the barrier and stores after it, and an
// object only moves to a lower position, so no store overwrites an object
// that is still to be read.  pre[i] = kept objects before position i of the
// shard, pre[n] = all kept; the flags are cleared for the next pass.
template <int KIND, class Rec>
__global__ __launch_bounds__(BLOCK) void k_cap_compact(EvDev E)
{
    __shared__ uint32_t s_sum[WAVES];
    if (upstream_overflow(E)) return;
    const int sh = blockIdx.x;
    const uint32_t rc = E.rc[KIND];
    const uint32_t c = E.gc[gc_shard(KIND, sh)];
    const uint32_t n = c < rc ? c : rc;
    const int32_t base = (int32_t)((uint32_t)sh * rc);
    int32_t *pre = E.cap_pre + (size_t)sh * (rc + 1);
    const int w = (int)(threadIdx.x >> 6), l = cap_lane();
    uint32_t run = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += BLOCK) {
        const uint32_t i = c0 + threadIdx.x;
        const bool live = i < n;
        bool keep = false;
        Rec r{};
        if (live) {
            keep = E.cap_drop[base + i] == 0;
            E.cap_drop[base + i] = 0;
            if (keep) r = rec_load(E, base + (int32_t)i, (Rec *)nullptr);
        }
        const unsigned long long m = __ballot(keep);
        const uint32_t below = (uint32_t)__popcll(m & ((1ull << l) - 1ull));
        if (l == 0) s_sum[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t wex = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < WAVES; ++q) {
            wex += q < w ? s_sum[q] : 0u;
            tot += s_sum[q];
        }
        const uint32_t at = run + wex + below;
        if (live) pre[i] = (int32_t)at;
        if (keep) rec_store(E, base + (int32_t)at, r);
        run += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pre[n] = (int32_t)run;
        E.gc[gc_shard(KIND, sh)] = run;
    }
}

// ---------------------------------------------------------------- fix ranges
__device__ __forceinline__ void remap(const EvDev &E, uint32_t rc, int32_t &start, int32_t &cnt)
{
    if (cnt <= 0) return;
    const int32_t sh = start / (int32_t)rc, loc = start - sh * (int32_t)rc;
    const int32_t *pre = E.cap_pre + (size_t)sh * (rc + 1);
    const int32_t a = pre[loc], b = pre[loc + cnt];
    start = sh * (int32_t)rc + a;
    cnt = b - a;
}

__global__ __launch_bounds__(BLOCK) void k_cap_fix_md(EvDev E)
{
    if (upstream_overflow(E)) return;
    const int n_slots = E.desc[D_NSLOTS];
    const uint32_t rc = E.rc[OT_MD];
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < n_slots; s += gridDim.x * BLOCK) {
        int32_t st = E.md_start[s], c = E.md_cnt[s];
        if (c <= 0) continue;
        remap(E, rc, st, c);
        E.md_start[s] = st;
        E.md_cnt[s] = c;
    }
}

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_cap_fix(EvDev E)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n_md = obj_prefix(E, OT_MD, s_pre);
    const uint32_t rc = E.rc[KIND];
    int32_t *st = KIND == OT_SEG ? E.seg_start : KIND == OT_T3 ? E.t3_start : E.t5_start;
    int32_t *ct = KIND == OT_SEG ? E.seg_cnt : KIND == OT_T3 ? E.t3_cnt : E.t5_cnt;
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < n_md; v += gridDim.x * BLOCK) {
        const int32_t m = obj_at(E, OT_MD, s_pre, v);
        int32_t s = st[m], c = ct[m];
        if (c <= 0) continue;
        remap(E, rc, s, c);
        st[m] = s;
        ct[m] = c;
    }
}

// ---------------------------------------------------------------- launch
static int cap_grid(int64_t work, int per_block)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > GRID_MAX) g = GRID_MAX;
    return (int)g;
}

hipError_t launch_cap(const EvDev &E, int type, int32_t cap, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    const int g_slots = cap_grid(E.cap_slots, WAVES);        // one wave per slot
    const int g_fix = cap_grid(E.cap_slots, BLOCK);
    switch (type) {
    case OT_MD:
        hipLaunchKernelGGL(k_cap_rank_md, dim3(g_slots), dim3(BLOCK), 0, s, E, cap);
        hipLaunchKernelGGL((k_cap_compact<OT_MD, MdRec>), dim3(NSH), dim3(BLOCK), 0, s, E);
        hipLaunchKernelGGL(k_cap_fix_md, dim3(g_fix), dim3(BLOCK), 0, s, E);
        break;
    case OT_SEG:
        hipLaunchKernelGGL(k_cap_rank<OT_SEG>, dim3(g_slots), dim3(BLOCK), 0, s, E, cap);
        hipLaunchKernelGGL((k_cap_compact<OT_SEG, SegRec>), dim3(NSH), dim3(BLOCK), 0, s, E);
        hipLaunchKernelGGL(k_cap_fix<OT_SEG>, dim3(GRID_MAX / 4), dim3(BLOCK), 0, s, E);
        break;
    case OT_T3:
        hipLaunchKernelGGL(k_cap_rank<OT_T3>, dim3(g_slots), dim3(BLOCK), 0, s, E, cap);
        hipLaunchKernelGGL((k_cap_compact<OT_T3, T3Rec>), dim3(NSH), dim3(BLOCK), 0, s, E);
        hipLaunchKernelGGL(k_cap_fix<OT_T3>, dim3(GRID_MAX / 4), dim3(BLOCK), 0, s, E);
        break;
    default:
        hipLaunchKernelGGL(k_cap_rank<OT_T5>, dim3(g_slots), dim3(BLOCK), 0, s, E, cap);
        hipLaunchKernelGGL((k_cap_compact<OT_T5, T5Rec>), dim3(NSH), dim3(BLOCK), 0, s, E);
        hipLaunchKernelGGL(k_cap_fix<OT_T5>, dim3(GRID_MAX / 4), dim3(BLOCK), 0, s, E);
        break;
    }
    return hipGetLastError();
}

}  // namespace lst
