// Pixel objects and track candidates (Sec. 2.1 of the paper and its
// kernel-flow figure, Sec. 3): pixel line segments (pLS, seeds of four
// pixel hits) linked to the kept quintuplets (pT5) and to the triplets
// (pT3), cross-cleaning of the collections, and the track candidates.
//
// Readings of the paper taken here (it gives no formula):
//  - a pLS links to an object inside a window around its direction (tangent
//    at the beam line, cot theta) when the chain of its four pixel hits and
//    the object's anchors passes an r-phi chi2 about the circle through its
//    first hit and two anchors and an r-z chi2 about the straight line in
//    arc length (score = their sum);
//  - inside the pT5 collection, and then inside the pT3 collection built
//    from the pLS that no surviving pT5 uses, a candidate survives iff no
//    candidate sharing one of its hits (pixel or outer) has a smaller
//    (score, seed, hit tuple) key;
//  - cross-cleaning in the paper's order: pT3 near a pT5 in eta-phi or
//    sharing a hit with one; kept quintuplets near or sharing a hit with a
//    pT5 or cleaned pT3; unlinked pLS against all of them, then among
//    themselves (the smaller seed index keeps a shared pixel hit);
//  - track candidates: pT5, pT3, T5 and pLS left after cleaning.
//
// The collections are small (thousands per event), so every step is a
// plain data-parallel pass: one wave per seed scans the objects of its event
// from a per-event list, one thread per candidate for the rest.  Per-hit
// minima use 64-bit atomics on (score bits, seed); ties on that key are
// resolved by the hit tuples.
#include <algorithm>

#include "lst_access.hpp"
#include "lst_cuts.hpp"

namespace lst {

__device__ __forceinline__ int px_lane() { return threadIdx.x & 63; }

constexpr unsigned long long KEY_NONE = ~0ull;

__device__ __forceinline__ int32_t *pl(const EvDev &E, int32_t *base, int list, bool plus1)
{
    return base + (size_t)list * (E.cap_ev + (plus1 ? 1 : 0));
}

// ---------------------------------------------------------------- setup
// every per-event list count, the per-hit minima and flags, seed state
__global__ __launch_bounds__(BLOCK) void k_px_init(EvDev E)
{
    if (upstream_overflow(E)) return;
    const int t0 = blockIdx.x * BLOCK + threadIdx.x, st = gridDim.x * BLOCK;
    const int n_ev = E.desc[D_NEV], n_px = E.desc[D_NPX], n_sd = E.desc[D_NSEEDS];
    const int n_hits = (int)E.gc[GC_N_SORTED];
    for (int i = t0; i < PXL_COUNT * E.cap_ev; i += st) {
        E.pl_cnt[i] = 0;
        E.pl_fill[i] = 0;
    }
    (void)n_ev;
    for (int i = t0; i < n_hits; i += st) {
        E.hmin_o[i] = KEY_NONE;
        E.hflag_o[i] = 0;
    }
    for (int i = t0; i < n_px; i += st) {
        E.hmin_p[i] = KEY_NONE;
        E.htie_p[i] = 0;
        E.hflag_p[i] = 0;
    }
    for (int i = t0; i < n_sd; i += st) {
        E.sd_used[i] = 0;
        E.sd_keep[i] = 0;
    }
}

// reset of the per-hit minima between two duplicate removals
__global__ __launch_bounds__(BLOCK) void k_px_rekey(EvDev E)
{
    if (upstream_overflow(E)) return;
    const int t0 = blockIdx.x * BLOCK + threadIdx.x, st = gridDim.x * BLOCK;
    const int n_px = E.desc[D_NPX], n_hits = (int)E.gc[GC_N_SORTED];
    for (int i = t0; i < n_hits; i += st) E.hmin_o[i] = KEY_NONE;
    for (int i = t0; i < n_px; i += st) {
        E.hmin_p[i] = KEY_NONE;
        E.htie_p[i] = 0;
    }
}

// seed directions
__global__ __launch_bounds__(BLOCK) void k_sd_dir(EvDev E)
{
    if (upstream_overflow(E)) return;
    const int n_sd = E.desc[D_NSEEDS];
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < n_sd; s += gridDim.x * BLOCK) {
        const int32_t a = E.sd_hits[4 * s], d = E.sd_hits[4 * s + 3];
        E.sd_dir[s] = pls_dir(E.px_x[a], E.px_y[a], E.px_z[a], E.px_x[d], E.px_y[d], E.px_z[d]);
    }
}

__device__ __forceinline__ int md_event(const EvDev &E, int32_t md, int n_mod)
{
    return E.md_slot[md] / n_mod;
}

// directions of the kept quintuplets and of every triplet, counted per event
__global__ __launch_bounds__(BLOCK) void k_obj_dir(EvDev E, int n_mod)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n5 = obj_prefix(E, OT_T5, s_pre);
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < n5; v += gridDim.x * BLOCK) {
        const int32_t t = obj_at(E, OT_T5, s_pre, v);
        if (!E.t5_keep[t]) continue;
        const MdV A = load_md(E, E.t5_md0[t]), C = load_md(E, E.t5_md2[t]), Q = load_md(E, E.t5_md4[t]);
        E.t5_dir[t] = obj_dir(A, Q, bridge_curv(A, C, Q));
        atomicAdd(&pl(E, E.pl_cnt, PXL_K5, false)[md_event(E, E.t5_md0[t], n_mod)], 1);
    }
    __syncthreads();
    const uint32_t n3 = obj_prefix(E, OT_T3, s_pre);
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < n3; v += gridDim.x * BLOCK) {
        const int32_t t = obj_at(E, OT_T3, s_pre, v);
        E.t3_dir[t] = obj_dir(load_md(E, E.t3_a[t]), load_md(E, E.t3_c[t]), E.t3_k[t]);
        atomicAdd(&pl(E, E.pl_cnt, PXL_K3, false)[md_event(E, E.t3_a[t], n_mod)], 1);
    }
}

// exclusive scan of one list's per-event counts (one block)
__global__ __launch_bounds__(1024) void k_pl_scan(EvDev E, int list)
{
    __shared__ int32_t s_part[1024];
    if (upstream_overflow(E)) return;
    const int n_ev = E.desc[D_NEV];
    const int32_t *cnt = pl(E, E.pl_cnt, list, false);
    int32_t *off = pl(E, E.pl_off, list, true);
    const int per = (n_ev + 1023) / 1024;
    const int a = threadIdx.x * per, b = min(a + per, n_ev);
    int32_t sum = 0;
    for (int e = a; e < b; ++e) sum += cnt[e];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < 1024; ++i) {
            const int32_t v = s_part[i];
            s_part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    int32_t run = s_part[threadIdx.x];
    for (int e = a; e < b; ++e) {
        off[e] = run;
        run += cnt[e];
    }
    if (b == n_ev && a <= b && (a < b || threadIdx.x == 0)) off[n_ev] = run;
}

// kept quintuplets and triplets into their per-event lists
__global__ __launch_bounds__(BLOCK) void k_obj_fill(EvDev E, int n_mod)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n5 = obj_prefix(E, OT_T5, s_pre);
    const int32_t *o5 = pl(E, E.pl_off, PXL_K5, true);
    int32_t *f5 = pl(E, E.pl_fill, PXL_K5, false);
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < n5; v += gridDim.x * BLOCK) {
        const int32_t t = obj_at(E, OT_T5, s_pre, v);
        if (!E.t5_keep[t]) continue;
        const int ev = md_event(E, E.t5_md0[t], n_mod);
        E.pl_k5[o5[ev] + atomicAdd(&f5[ev], 1)] = t;
    }
    __syncthreads();
    const uint32_t n3 = obj_prefix(E, OT_T3, s_pre);
    const int32_t *o3 = pl(E, E.pl_off, PXL_K3, true);
    int32_t *f3 = pl(E, E.pl_fill, PXL_K3, false);
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < n3; v += gridDim.x * BLOCK) {
        const int32_t t = obj_at(E, OT_T3, s_pre, v);
        const int ev = md_event(E, E.t3_a[t], n_mod);
        E.pl_k3[o3[ev] + atomicAdd(&f3[ev], 1)] = t;
    }
}

// ---------------------------------------------------------------- linking
// the MDs of an outer object, inner to outer
template <int KIND>
__device__ __forceinline__ int32_t obj_md(const EvDev &E, int32_t t, int j)
{
    if constexpr (KIND == 5) return t5_md(E, t, j);
    else return j == 0 ? E.t3_a[t] : j == 1 ? E.t3_b[t] : E.t3_c[t];
}

// One wave per seed: the objects of its event 64 at a time; window, then the
// link chi2 on the lanes inside it; accepted candidates appended with one
// atomic per chunk.
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_px_link(EvDev E, Consts K, PixConsts P)
{
    constexpr int NP = 4 + KIND, IC = KIND == 5 ? 6 : 4;
    const int l = px_lane();
    const int n_sd = E.desc[D_NSEEDS];
    const int nw = gridDim.x * WAVES;
    const int32_t *off = pl(E, E.pl_off, KIND == 5 ? PXL_K5 : PXL_K3, true);
    const int32_t *lst = KIND == 5 ? E.pl_k5 : E.pl_k3;
    const float4 *dir = KIND == 5 ? E.t5_dir : E.t3_dir;
    int32_t *c_seed = KIND == 5 ? E.c5_seed : E.c3_seed;
    int32_t *c_obj = KIND == 5 ? E.c5_obj : E.c3_obj;
    float *c_score = KIND == 5 ? E.c5_score : E.c3_score;
    const float x2p = KIND == 5 ? P.x5p : P.x3p, x2z = KIND == 5 ? P.x5z : P.x3z;
    const unsigned long long below = (1ull << l) - 1ull;
    if (upstream_overflow(E)) return;
    for (int s = blockIdx.x * WAVES + (int)(threadIdx.x >> 6); s < n_sd; s += nw) {
        if (KIND == 3 && E.sd_used[s]) continue;
        const int ev = E.sd_ev[s];
        const float4 d = E.sd_dir[s];
        LPt pix[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t h = E.sd_hits[4 * s + k];
            pix[k] = lpt_px(E.px_x[h], E.px_y[h], E.px_z[h]);
        }
        const int32_t b0 = off[ev], b1 = off[ev + 1];
        for (int32_t b = b0; b < b1; b += 64) {
            const int32_t i = b + l;
            bool ok = false;
            float score = 0.0f;
            int32_t t = 0;
            if (i < b1) {
                t = lst[i];
                if (link_window(d, dir[t], P.wl2)) {
                    LPt pts[NP];
#pragma unroll
                    for (int k = 0; k < 4; ++k) pts[k] = pix[k];
#pragma unroll
                    for (int j = 0; j < KIND; ++j) pts[4 + j] = lpt_md(load_md(E, obj_md<KIND>(E, t, j)));
                    ok = link_accept<NP, IC>(K, pts, P.sig2p, P.sigz, x2p, x2z, score);
                }
            }
            const unsigned long long m = __ballot(ok);
            if (m) {
                uint32_t base = 0;
                if (l == 0) base = atomicAdd(&E.gc[KIND == 5 ? GC_PX5 : GC_PX3], (uint32_t)__popcll(m));
                base = __shfl(base, 0, 64);
                if (ok) {
                    const uint32_t at = base + (uint32_t)__popcll(m & below);
                    if (at < (uint32_t)E.cap_pxc) {
                        c_seed[at] = s;
                        c_obj[at] = t;
                        c_score[at] = score;
                    } else {
                        atomicOr(&E.gc[GC_OVERFLOW], 1u << OT_COUNT);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- duplicate removal
template <int KIND>
__device__ __forceinline__ unsigned long long c_key(const EvDev &E, uint32_t c)
{
    const float sc = KIND == 5 ? E.c5_score[c] : E.c3_score[c];
    const int32_t s = KIND == 5 ? E.c5_seed[c] : E.c3_seed[c];
    return ((unsigned long long)__float_as_uint(sc) << 32) | (uint32_t)E.sd_local[s];
}

template <int KIND>
__device__ __forceinline__ uint32_t n_cand(const EvDev &E)
{
    const uint32_t n = E.gc[KIND == 5 ? GC_PX5 : GC_PX3];
    return n < (uint32_t)E.cap_pxc ? n : (uint32_t)E.cap_pxc;
}

// grouped position of outer hit j (0 .. 2 KIND - 1) of candidate c's object
template <int KIND>
__device__ __forceinline__ int32_t c_ohit(const EvDev &E, int32_t obj, int j)
{
    const int32_t m = obj_md<KIND>(E, obj, j >> 1);
    return (j & 1) ? E.md_hup[m] : E.md_hlo[m];
}

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_pxd_min(EvDev E)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<KIND>(E);
    for (uint32_t c = blockIdx.x * BLOCK + threadIdx.x; c < n; c += gridDim.x * BLOCK) {
        const unsigned long long key = c_key<KIND>(E, c);
        const int32_t s = KIND == 5 ? E.c5_seed[c] : E.c3_seed[c];
        const int32_t o = KIND == 5 ? E.c5_obj[c] : E.c3_obj[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) atomicMin(&E.hmin_p[E.sd_hits[4 * s + k]], key);
#pragma unroll
        for (int j = 0; j < 2 * KIND; ++j) atomicMin(&E.hmin_o[c_ohit<KIND>(E, o, j)], key);
    }
}

// candidates reaching the minimum of their first pixel hit: more than one
// means two candidates of one seed with equal scores
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_pxd_tie(EvDev E)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<KIND>(E);
    for (uint32_t c = blockIdx.x * BLOCK + threadIdx.x; c < n; c += gridDim.x * BLOCK) {
        const int32_t s = KIND == 5 ? E.c5_seed[c] : E.c3_seed[c];
        const int32_t p0 = E.sd_hits[4 * s];
        if (E.hmin_p[p0] == c_key<KIND>(E, c)) atomicAdd(&E.htie_p[p0], 1u);
    }
}

// per-event hit index of outer hit j of an object
template <int KIND>
__device__ __forceinline__ int32_t c_orig(const EvDev &E, int32_t obj, int j)
{
    return __float_as_int(E.hsort[c_ohit<KIND>(E, obj, j)].w);
}

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_pxd_keep(EvDev E, int n_mod)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<KIND>(E);
    for (uint32_t c = blockIdx.x * BLOCK + threadIdx.x; c < n; c += gridDim.x * BLOCK) {
        const unsigned long long key = c_key<KIND>(E, c);
        const int32_t s = KIND == 5 ? E.c5_seed[c] : E.c3_seed[c];
        const int32_t o = KIND == 5 ? E.c5_obj[c] : E.c3_obj[c];
        bool keep = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) keep = keep && E.hmin_p[E.sd_hits[4 * s + k]] == key;
#pragma unroll
        for (int j = 0; j < 2 * KIND; ++j) keep = keep && E.hmin_o[c_ohit<KIND>(E, o, j)] == key;
        if (keep && E.htie_p[E.sd_hits[4 * s]] > 1u) {
            // equal (score, seed): the smaller outer hit tuple wins
            const float sc = KIND == 5 ? E.c5_score[c] : E.c3_score[c];
            for (uint32_t u = 0; u < n && keep; ++u) {
                if (u == c) continue;
                const int32_t su = KIND == 5 ? E.c5_seed[u] : E.c3_seed[u];
                const float scu = KIND == 5 ? E.c5_score[u] : E.c3_score[u];
                if (su != s || __float_as_uint(scu) != __float_as_uint(sc)) continue;
                const int32_t ou = KIND == 5 ? E.c5_obj[u] : E.c3_obj[u];
                for (int j = 0; j < 2 * KIND; ++j) {
                    const int32_t a = c_orig<KIND>(E, ou, j), b = c_orig<KIND>(E, o, j);
                    if (a != b) {
                        if (a < b) keep = false;
                        break;
                    }
                }
            }
        }
        if (KIND == 5) {
            E.c5_keep[c] = keep;
            if (keep) {
                E.sd_used[s] = 1;
                atomicAdd(&pl(E, E.pl_cnt, PXL_D5, false)[E.sd_ev[s]], 1);
            }
        } else {
            E.c3_keep[c] = keep;
        }
    }
    (void)n_mod;
}

// ---------------------------------------------------------------- cross-cleaning
__device__ __forceinline__ bool near_any(const EvDev &E, int list, int ev, const float4 *dirs,
                                         const float4 &d, float dr2)
{
    const int32_t *off = pl(E, E.pl_off, list, true);
    for (int32_t i = off[ev]; i < off[ev + 1]; ++i)
        if (close_dir(d, dirs[i], dr2)) return true;
    return false;
}

// surviving pT5: their directions into the event list, their hits flagged
__global__ __launch_bounds__(BLOCK) void k_pt5_mark(EvDev E)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<5>(E);
    const int32_t *off = pl(E, E.pl_off, PXL_D5, true);
    int32_t *fill = pl(E, E.pl_fill, PXL_D5, false);
    for (uint32_t c = blockIdx.x * BLOCK + threadIdx.x; c < n; c += gridDim.x * BLOCK) {
        if (!E.c5_keep[c]) continue;
        const int32_t s = E.c5_seed[c], o = E.c5_obj[c];
        const int ev = E.sd_ev[s];
        E.pl_d5[off[ev] + atomicAdd(&fill[ev], 1)] = E.sd_dir[s];
        for (int k = 0; k < 4; ++k) E.hflag_p[E.sd_hits[4 * s + k]] = 1;
        for (int j = 0; j < 10; ++j) E.hflag_o[c_ohit<5>(E, o, j)] = 1;
    }
}

// pT3 near a pT5 or sharing a hit with one are duplicates
__global__ __launch_bounds__(BLOCK) void k_pt3_clean(EvDev E, PixConsts P)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<3>(E);
    for (uint32_t c = blockIdx.x * BLOCK + threadIdx.x; c < n; c += gridDim.x * BLOCK) {
        if (!E.c3_keep[c]) continue;
        const int32_t s = E.c3_seed[c], o = E.c3_obj[c];
        bool keep = true;
        for (int k = 0; k < 4; ++k) keep = keep && !E.hflag_p[E.sd_hits[4 * s + k]];
        for (int j = 0; j < 6; ++j) keep = keep && !E.hflag_o[c_ohit<3>(E, o, j)];
        if (keep) keep = !near_any(E, PXL_D5, E.sd_ev[s], E.pl_d5, E.sd_dir[s], P.dr2);
        E.c3_keep[c] = keep;
        if (keep) atomicAdd(&pl(E, E.pl_cnt, PXL_D3, false)[E.sd_ev[s]], 1);
    }
}

// cleaned pT3: directions into the event list, hits flagged, seeds used
__global__ __launch_bounds__(BLOCK) void k_pt3_mark(EvDev E)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<3>(E);
    const int32_t *off = pl(E, E.pl_off, PXL_D3, true);
    int32_t *fill = pl(E, E.pl_fill, PXL_D3, false);
    for (uint32_t c = blockIdx.x * BLOCK + threadIdx.x; c < n; c += gridDim.x * BLOCK) {
        if (!E.c3_keep[c]) continue;
        const int32_t s = E.c3_seed[c], o = E.c3_obj[c];
        const int ev = E.sd_ev[s];
        E.pl_d3[off[ev] + atomicAdd(&fill[ev], 1)] = E.sd_dir[s];
        E.sd_used[s] = 1;
        for (int k = 0; k < 4; ++k) E.hflag_p[E.sd_hits[4 * s + k]] = 1;
        for (int j = 0; j < 6; ++j) E.hflag_o[c_ohit<3>(E, o, j)] = 1;
    }
}

// kept quintuplets near, or sharing a hit with, a pT5 or cleaned pT3
__global__ __launch_bounds__(BLOCK) void k_t5_clean(EvDev E, PixConsts P, int n_mod)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n5 = obj_prefix(E, OT_T5, s_pre);
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < n5; v += gridDim.x * BLOCK) {
        const int32_t t = obj_at(E, OT_T5, s_pre, v);
        bool keep = E.t5_keep[t] != 0;
        if (keep) {
            for (int j = 0; j < 10; ++j) keep = keep && !E.hflag_o[c_ohit<5>(E, t, j)];
            const int ev = md_event(E, E.t5_md0[t], n_mod);
            const float4 d = E.t5_dir[t];
            if (keep) keep = !near_any(E, PXL_D5, ev, E.pl_d5, d, P.dr2);
            if (keep) keep = !near_any(E, PXL_D3, ev, E.pl_d3, d, P.dr2);
            if (keep) atomicAdd(&pl(E, E.pl_cnt, PXL_DT, false)[ev], 1);
        }
        E.t5_clean[t] = keep;
    }
}

__global__ __launch_bounds__(BLOCK) void k_t5_clean_fill(EvDev E, int n_mod)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n5 = obj_prefix(E, OT_T5, s_pre);
    const int32_t *off = pl(E, E.pl_off, PXL_DT, true);
    int32_t *fill = pl(E, E.pl_fill, PXL_DT, false);
    for (uint32_t v = blockIdx.x * BLOCK + threadIdx.x; v < n5; v += gridDim.x * BLOCK) {
        const int32_t t = obj_at(E, OT_T5, s_pre, v);
        if (!E.t5_clean[t]) continue;
        const int ev = md_event(E, E.t5_md0[t], n_mod);
        E.pl_dt[off[ev] + atomicAdd(&fill[ev], 1)] = E.t5_dir[t];
    }
}

// unlinked pLS: a pixel hit held by a candidate, or near one, is a
// duplicate; the rest mark their pixel hits with their index (minimum)
__global__ __launch_bounds__(BLOCK) void k_pls_clean(EvDev E, PixConsts P)
{
    if (upstream_overflow(E)) return;
    const int n_sd = E.desc[D_NSEEDS];
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < n_sd; s += gridDim.x * BLOCK) {
        if (E.sd_used[s]) continue;
        bool keep = true;
        for (int k = 0; k < 4; ++k) keep = keep && !E.hflag_p[E.sd_hits[4 * s + k]];
        const int ev = E.sd_ev[s];
        const float4 d = E.sd_dir[s];
        if (keep) keep = !near_any(E, PXL_D5, ev, E.pl_d5, d, P.dr2);
        if (keep) keep = !near_any(E, PXL_D3, ev, E.pl_d3, d, P.dr2);
        if (keep) keep = !near_any(E, PXL_DT, ev, E.pl_dt, d, P.dr2);
        E.sd_keep[s] = keep;
        if (keep)
            for (int k = 0; k < 4; ++k)
                atomicMin(&E.hmin_p[E.sd_hits[4 * s + k]], (unsigned long long)(uint32_t)E.sd_local[s]);
    }
}

__global__ __launch_bounds__(BLOCK) void k_pls_keep(EvDev E)
{
    if (upstream_overflow(E)) return;
    const int n_sd = E.desc[D_NSEEDS];
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < n_sd; s += gridDim.x * BLOCK) {
        if (!E.sd_keep[s]) continue;
        const unsigned long long me = (unsigned long long)(uint32_t)E.sd_local[s];
        bool keep = true;
        for (int k = 0; k < 4; ++k) keep = keep && E.hmin_p[E.sd_hits[4 * s + k]] == me;
        E.sd_keep[s] = keep;
    }
}

// ---------------------------------------------------------------- launch
static int px_grid(int64_t work, int per_block)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > GRID_MAX) g = GRID_MAX;
    return (int)g;
}

hipError_t launch_pixel(const EvDev &E, const Consts &K, const PixConsts &P, hipStream_t s)
{
    const int n_mod = E.cap_slots / E.cap_ev;
    const int g_hits = px_grid(std::max<int64_t>(E.cap_hits, E.cap_px), BLOCK);
    const int g_sd = px_grid(E.cap_seeds, BLOCK);
    const int g_sdw = px_grid(E.cap_seeds, WAVES);
    const int g_c = px_grid(E.cap_pxc, BLOCK);
    const int g_obj = px_grid((int64_t)E.rc[OT_T3] * NSH, BLOCK);
    hipLaunchKernelGGL(k_px_init, dim3(g_hits), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_sd_dir, dim3(g_sd), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_obj_dir, dim3(g_obj), dim3(BLOCK), 0, s, E, n_mod);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_K5);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_K3);
    hipLaunchKernelGGL(k_obj_fill, dim3(g_obj), dim3(BLOCK), 0, s, E, n_mod);
    // pT5
    hipLaunchKernelGGL(k_px_link<5>, dim3(g_sdw), dim3(BLOCK), 0, s, E, K, P);
    hipLaunchKernelGGL(k_pxd_min<5>, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_pxd_tie<5>, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_pxd_keep<5>, dim3(g_c), dim3(BLOCK), 0, s, E, n_mod);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_D5);
    hipLaunchKernelGGL(k_pt5_mark, dim3(g_c), dim3(BLOCK), 0, s, E);
    // pT3 from the seeds no pT5 uses
    hipLaunchKernelGGL(k_px_rekey, dim3(g_hits), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_px_link<3>, dim3(g_sdw), dim3(BLOCK), 0, s, E, K, P);
    hipLaunchKernelGGL(k_pxd_min<3>, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_pxd_tie<3>, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_pxd_keep<3>, dim3(g_c), dim3(BLOCK), 0, s, E, n_mod);
    // cross-cleaning
    hipLaunchKernelGGL(k_pt3_clean, dim3(g_c), dim3(BLOCK), 0, s, E, P);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_D3);
    hipLaunchKernelGGL(k_pt3_mark, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_t5_clean, dim3(g_obj), dim3(BLOCK), 0, s, E, P, n_mod);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_DT);
    hipLaunchKernelGGL(k_t5_clean_fill, dim3(g_obj), dim3(BLOCK), 0, s, E, n_mod);
    hipLaunchKernelGGL(k_px_rekey, dim3(g_hits), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_pls_clean, dim3(g_sd), dim3(BLOCK), 0, s, E, P);
    hipLaunchKernelGGL(k_pls_keep, dim3(g_sd), dim3(BLOCK), 0, s, E);
    return hipGetLastError();
}

}  // namespace lst
