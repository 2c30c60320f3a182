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
// from a per-event list, one wave per object scans the direction lists of
// its event in the cross-cleaning, one thread per candidate for the rest.
// Per-hit minima use 64-bit atomics on (score bits, seed); ties on that key
// are resolved by the hit tuples.  List counters take one atomic per wave
// and list key (one address taking an atomic per object would
// serialise thousands of device-scope atomics).  Every per-event list is
// kept per (event, azimuth bin), so that a seed or an object scans only the
// bins its window or closeness reaches.
#include <algorithm>

#include "lst_access.hpp"
#include "lst_cuts.hpp"

namespace lst {

__device__ __forceinline__ int px_lane() { return threadIdx.x & 63; }

constexpr unsigned long long KEY_NONE = ~0ull;

// list `list` of pl_cnt / pl_off / pl_fill
__device__ __forceinline__ int32_t *pl(const EvDev &E, int32_t *base, int list)
{
    return base + (size_t)list * ((size_t)E.cap_ev * PX_NB + 1);
}

// azimuth bin of a direction (tangent t.x, t.y): floor((phi + pi) PX_NB /
// 2 pi), clamped; monotone in phi
constexpr float PX_PI = 3.14159265358979f;
__device__ __forceinline__ int phi_bin(float phi)
{
    const float b = (phi + PX_PI) * (PX_NB / (2.0f * PX_PI));
    return b > 0.0f ? (int)fminf(b, (float)(PX_NB - 1)) : 0;
}

__device__ __forceinline__ int dir_bin(const float4 &d) { return phi_bin(atan2f(d.y, d.x)); }

// The bins holding every direction within wphi of d in azimuth: [a0, b0]
// and, across the wrap at +-pi, [a1, b1] (empty when a1 > b1).  A NaN
// direction passes no window; it scans every bin.
__device__ __forceinline__ void window_bins(const float4 &d, float wphi, int &a0, int &b0, int &a1,
                                            int &b1)
{
    a0 = 0;
    b0 = PX_NB - 1;
    a1 = 1;
    b1 = 0;
    const float ph = atan2f(d.y, d.x);
    if (!(wphi < PX_PI) || !(ph == ph)) return;
    const float lo = ph - wphi, hi = ph + wphi;
    if (lo < -PX_PI) {
        b0 = phi_bin(hi);
        a1 = phi_bin(lo + 2.0f * PX_PI);
        b1 = PX_NB - 1;
    } else if (hi > PX_PI) {
        a0 = phi_bin(lo);
        a1 = 0;
        b1 = phi_bin(hi - 2.0f * PX_PI);
    } else {
        a0 = phi_bin(lo);
        b0 = phi_bin(hi);
    }
    // the two parts meet: every bin, once
    if (a1 <= b1 && (a1 <= b0 + 1 && b1 + 1 >= a0)) {
        a0 = 0;
        b0 = PX_NB - 1;
        a1 = 1;
        b1 = 0;
    }
}

// Add one to cnt[key] for every active lane with `act`: the lanes are
// grouped by key with ballots, then each group's first lane adds the group's
// size (the wave's atomics go out together: one memory round trip); returns
// each such lane's old value plus its rank in its group (its slot in a list
// being filled).
__device__ __forceinline__ int32_t agg_add(int32_t *cnt, int key, bool act)
{
    const int l = px_lane();
    const unsigned long long below = (1ull << l) - 1ull;
    int lead_of = l, rank = 0, size = 0;
    unsigned long long todo = __ballot(act);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int k = __shfl(key, lead, 64);
        const unsigned long long grp = todo & __ballot(key == k);
        if ((grp >> l) & 1ull) {
            lead_of = lead;
            rank = (int)__popcll(grp & below);
        }
        if (l == lead) size = (int)__popcll(grp);
        todo &= ~grp;
    }
    int32_t base = 0;
    if (size > 0) base = atomicAdd(&cnt[key], size);
    base = __shfl(base, lead_of, 64);
    return base + rank;
}

// Objects handed to one wave, consecutive, in the one-wave-per-object passes
constexpr int PX_WCHUNK = 2;

// A count per list key kept by one wave over its run of objects: one atomic
// when the key changes and one at the end.
struct EvRun {
    int ev = -1;
    int32_t n = 0;
    __device__ void add(int32_t *cnt, int e)
    {
        if (e != ev) {
            flush(cnt);
            ev = e;
        }
        ++n;
    }
    __device__ void flush(int32_t *cnt)
    {
        if (n > 0 && px_lane() == 0) atomicAdd(&cnt[ev], n);
        n = 0;
    }
};

// ---------------------------------------------------------------- setup
// every per-event list count, the per-hit minima and flags, seed state and
// direction
__global__ __launch_bounds__(BLOCK) void k_px_init(EvDev E)
{
    if (upstream_overflow(E)) return;
    const int t0 = blockIdx.x * BLOCK + threadIdx.x, st = gridDim.x * BLOCK;
    const int n_ev = E.desc[D_NEV], n_px = E.desc[D_NPX], n_sd = E.desc[D_NSEEDS];
    const int n_hits = (int)E.gc[GC_N_SORTED];
    const int n_pl = PXL_COUNT * (E.cap_ev * PX_NB + 1);
    for (int i = t0; i < n_pl; i += st) {
        E.pl_cnt[i] = 0;
        E.pl_fill[i] = 0;
    }
    for (int i = t0; i < n_sd; i += st) {
        E.sd_c5[i] = make_int2(0, 0);
        E.sd_c3[i] = make_int2(0, 0);
    }
    (void)n_ev;
    for (int i = t0; i < n_hits; i += st) {
        E.hmin_o[i] = KEY_NONE;
        E.hflag_o[i] = 0;
    }
    for (int i = t0; i < n_px; i += st) {
        E.hmin_p[i] = KEY_NONE;
        E.hflag_p[i] = 0;
    }
    for (int i = t0; i < n_sd; i += st) {
        E.sd_used[i] = 0;
        E.sd_keep[i] = 0;
        // seed direction
        const int32_t a = E.sd_hits[4 * i], d = E.sd_hits[4 * i + 3];
        E.sd_dir[i] = pls_dir(E.px_x[a], E.px_y[a], E.px_z[a], E.px_x[d], E.px_y[d], E.px_z[d]);
    }
}

// reset of the per-hit minima between two duplicate removals; with
// list_free, also the list of the seeds that no kept pT5 uses (run inside
// the kernels that precede the next users)
__device__ __forceinline__ void rekey_body(const EvDev &E, bool list_free)
{
    const int t0 = blockIdx.x * BLOCK + threadIdx.x, st = gridDim.x * BLOCK;
    const int n_px = E.desc[D_NPX], n_hits = (int)E.gc[GC_N_SORTED], n_sd = E.desc[D_NSEEDS];
    for (int i = t0; i < n_hits; i += st) E.hmin_o[i] = KEY_NONE;
    for (int i = t0; i < n_px; i += st) E.hmin_p[i] = KEY_NONE;
    if (!list_free) return;
    for (int s0 = blockIdx.x * BLOCK; s0 < n_sd; s0 += st) {
        const int s = s0 + (int)threadIdx.x;
        const bool act = s < n_sd && !E.sd_used[s];
        const int32_t at = agg_add(reinterpret_cast<int32_t *>(E.gc + GC_PXFREE), 0, act);
        if (act) E.sd_free[at] = s;
    }
}

__device__ __forceinline__ int md_event(const EvDev &E, int32_t md, int n_mod)
{
    return E.md_slot[md] / n_mod;
}

// directions of the kept quintuplets and of every triplet, counted per
// (event, azimuth bin)
__global__ __launch_bounds__(BLOCK) void k_obj_dir(EvDev E, int n_mod)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n5 = obj_prefix(E, OT_T5, s_pre);
    for (uint32_t v0 = blockIdx.x * BLOCK; v0 < n5; v0 += gridDim.x * BLOCK) {
        const uint32_t v = v0 + threadIdx.x;
        bool act = false;
        int ev = 0;
        if (v < n5) {
            const int32_t t = obj_at(E, OT_T5, s_pre, v);
            if (E.t5_keep[t]) {
                const MdV A = load_md(E, E.t5_md0[t]), C = load_md(E, E.t5_md2[t]),
                          Q = load_md(E, E.t5_md4[t]);
                const float4 d = obj_dir(A, Q, bridge_curv(A, C, Q));
                E.t5_dir[t] = d;
                ev = md_event(E, E.t5_md0[t], n_mod) * PX_NB + dir_bin(d);
                act = true;
            }
        }
        (void)agg_add(pl(E, E.pl_cnt, PXL_K5), ev, act);
    }
    __syncthreads();
    const uint32_t n3 = obj_prefix(E, OT_T3, s_pre);
    for (uint32_t v0 = blockIdx.x * BLOCK; v0 < n3; v0 += gridDim.x * BLOCK) {
        const uint32_t v = v0 + threadIdx.x;
        int ev = 0;
        if (v < n3) {
            const int32_t t = obj_at(E, OT_T3, s_pre, v);
            const float4 d = obj_dir(load_md(E, E.t3_a[t]), load_md(E, E.t3_c[t]), E.t3_k[t]);
            E.t3_dir[t] = d;
            ev = md_event(E, E.t3_a[t], n_mod) * PX_NB + dir_bin(d);
        }
        (void)agg_add(pl(E, E.pl_cnt, PXL_K3), ev, v < n3);
    }
}

// exclusive scan of a list's counts, n_ev x mult keys (block 0: list0,
// block 1: list1); off[n] = the total
__global__ __launch_bounds__(1024) void k_pl_scan(EvDev E, int list0, int list1, int mult)
{
    __shared__ int32_t s_part[1024];
    if (upstream_overflow(E)) return;
    const int list = blockIdx.x == 0 ? list0 : list1;
    const int n = E.desc[D_NEV] * mult;
    const int32_t *cnt = pl(E, E.pl_cnt, list);
    int32_t *off = pl(E, E.pl_off, list);
    const int per = (n + 1023) / 1024;
    const int a = threadIdx.x * per, b = min(a + per, n);
    int32_t sum = 0;
    for (int e = a; e < b; ++e) sum += cnt[e];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    // inclusive scan of the 1024 partial sums (doubling steps)
    for (int d = 1; d < 1024; d <<= 1) {
        const int32_t add = (int)threadIdx.x >= d ? s_part[threadIdx.x - d] : 0;
        __syncthreads();
        s_part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = s_part[threadIdx.x] - sum;
    for (int e = a; e < b; ++e) {
        off[e] = run;
        run += cnt[e];
    }
    if (threadIdx.x == 1023) off[n] = s_part[1023];
}

// kept quintuplets and triplets into their per-(event, bin) lists
__global__ __launch_bounds__(BLOCK) void k_obj_fill(EvDev E, int n_mod)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n5 = obj_prefix(E, OT_T5, s_pre);
    const int32_t *o5 = pl(E, E.pl_off, PXL_K5);
    int32_t *f5 = pl(E, E.pl_fill, PXL_K5);
    for (uint32_t v0 = blockIdx.x * BLOCK; v0 < n5; v0 += gridDim.x * BLOCK) {
        const uint32_t v = v0 + threadIdx.x;
        int32_t t = 0;
        int ev = 0;
        bool act = false;
        if (v < n5) {
            t = obj_at(E, OT_T5, s_pre, v);
            act = E.t5_keep[t] != 0;
            if (act) ev = md_event(E, E.t5_md0[t], n_mod) * PX_NB + dir_bin(E.t5_dir[t]);
        }
        const int32_t at = agg_add(f5, ev, act);
        if (act) {
            E.pl_k5[o5[ev] + at] = t;
            E.pl_k5d[o5[ev] + at] = E.t5_dir[t];
        }
    }
    __syncthreads();
    const uint32_t n3 = obj_prefix(E, OT_T3, s_pre);
    const int32_t *o3 = pl(E, E.pl_off, PXL_K3);
    int32_t *f3 = pl(E, E.pl_fill, PXL_K3);
    for (uint32_t v0 = blockIdx.x * BLOCK; v0 < n3; v0 += gridDim.x * BLOCK) {
        const uint32_t v = v0 + threadIdx.x;
        int32_t t = 0;
        int ev = 0;
        if (v < n3) {
            t = obj_at(E, OT_T3, s_pre, v);
            ev = md_event(E, E.t3_a[t], n_mod) * PX_NB + dir_bin(E.t3_dir[t]);
        }
        const int32_t at = agg_add(f3, ev, v < n3);
        if (v < n3) {
            E.pl_k3[o3[ev] + at] = t;
            E.pl_k3d[o3[ev] + at] = E.t3_dir[t];
        }
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

// grouped position of outer hit j (0 .. 2 KIND - 1) of candidate c's object
template <int KIND>
__device__ __forceinline__ int32_t c_ohit(const EvDev &E, int32_t obj, int j)
{
    const int32_t m = obj_md<KIND>(E, obj, j >> 1);
    return (j & 1) ? E.md_hup[m] : E.md_hlo[m];
}

// WPS waves per seed: the objects of its event in the azimuth bins of its
// link window, 64 at a time (wave q of the seed takes every WPS-th chunk);
// window, then the link chi2 on the lanes inside it.  A block of PX_LW
// waves takes PX_LW / WPS seeds per round (pT5: every seed; pT3: the seeds
// that no kept pT5 uses, from their list), stages the accepted candidates in
// LDS and reserves room for the round's candidates with one atomic, so each
// seed's candidates are consecutive (its range in sd_c5 / sd_c3).  A wave
// with more than PX_STAGE candidates scans again and writes the rest
// directly.
constexpr int PX_LW = 16, PX_STAGE = 64;

struct SmLink {
    int32_t obj[PX_LW][PX_STAGE];
    float score[PX_LW][PX_STAGE];
    uint32_t cnt[PX_LW], base;
};

template <int KIND, int WPS>
__device__ __forceinline__ void link_scan(const EvDev &E, const Consts &K, const PixConsts &P,
                                          int s, int ev, const float4 &d, const LPt *pix, int q,
                                          uint32_t &n_acc, SmLink &sm, int w, uint32_t write_base,
                                          bool second)
{
    constexpr int NP = 4 + KIND, IC = KIND == 5 ? 6 : 4;
    const int l = px_lane();
    const unsigned long long below = (1ull << l) - 1ull;
    const int32_t *off = pl(E, E.pl_off, KIND == 5 ? PXL_K5 : PXL_K3);
    const int32_t *lst = KIND == 5 ? E.pl_k5 : E.pl_k3;
    const float4 *dir = KIND == 5 ? E.pl_k5d : E.pl_k3d;   // in list order
    const float x2p = KIND == 5 ? P.x5p : P.x3p, x2z = KIND == 5 ? P.x5z : P.x3z;
    int a[2], b[2];
    window_bins(d, P.wphi, a[0], b[0], a[1], b[1]);
    for (int part = 0; part < 2; ++part) {
        if (a[part] > b[part]) continue;
        const int32_t i0 = off[ev * PX_NB + a[part]] + 64 * q, i1 = off[ev * PX_NB + b[part] + 1];
        // the next chunk's entries are loaded while this one is tested
        int32_t tn = 0;
        float4 dn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (i0 + l < i1) {
            tn = lst[i0 + l];
            dn = dir[i0 + l];
        }
        for (int32_t i = i0 + l, base = i0; base < i1; base += 64 * WPS, i += 64 * WPS) {
            const int32_t t = tn;
            const float4 dt = dn;
            if (i + 64 * WPS < i1) {
                tn = lst[i + 64 * WPS];
                dn = dir[i + 64 * WPS];
            }
            bool ok = false;
            float score = 0.0f;
            if (i < i1 && link_window(d, dt, P.wl2)) {
                LPt pts[NP];
#pragma unroll
                for (int k = 0; k < 4; ++k) pts[k] = pix[k];
#pragma unroll
                for (int j = 0; j < KIND; ++j) pts[4 + j] = lpt_md(load_md(E, obj_md<KIND>(E, t, j)));
                ok = link_accept<NP, IC>(K, pts, P.sig2p, P.sigz, x2p, x2z, score);
            }
            const unsigned long long m = __ballot(ok);
            if (ok) {
                const uint32_t pos = n_acc + (uint32_t)__popcll(m & below);
                if (!second && pos < PX_STAGE) {
                    sm.obj[w][pos] = t;
                    sm.score[w][pos] = score;
                } else if (second && pos >= PX_STAGE) {
                    const uint32_t at = write_base + pos;
                    if (at < (uint32_t)E.cap_pxc) {
                        (KIND == 5 ? E.c5_seed : E.c3_seed)[at] = s;
                        (KIND == 5 ? E.c5_obj : E.c3_obj)[at] = t;
                        (KIND == 5 ? E.c5_score : E.c3_score)[at] = score;
                    }
                }
            }
            n_acc += (uint32_t)__popcll(m);
        }
    }
}

template <int KIND, int WPS>
__global__ __launch_bounds__(PX_LW * 64) void k_px_link(EvDev E, Consts K, PixConsts P)
{
    static_assert(PX_LW % WPS == 0, "whole seeds per block");
    __shared__ SmLink sm;
    const int l = px_lane(), w = (int)(threadIdx.x >> 6), q = w % WPS;
    const int n = KIND == 5 ? E.desc[D_NSEEDS] : (int)E.gc[GC_PXFREE];
    int32_t *c_seed = KIND == 5 ? E.c5_seed : E.c3_seed;
    int32_t *c_obj = KIND == 5 ? E.c5_obj : E.c3_obj;
    float *c_score = KIND == 5 ? E.c5_score : E.c3_score;
    int2 *sd_c = KIND == 5 ? E.sd_c5 : E.sd_c3;
    constexpr int SPB = PX_LW / WPS;   // seeds per block and round
    if (upstream_overflow(E)) return;
    for (int r0 = blockIdx.x * SPB; r0 < n; r0 += gridDim.x * SPB) {
        const int v = r0 + w / WPS;
        const bool act = v < n;
        const int s = act ? (KIND == 5 ? v : E.sd_free[v]) : 0;
        uint32_t n_acc = 0;
        int ev = 0;
        float4 d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        LPt pix[4];
        if (act) {
            ev = E.sd_ev[s];
            d = E.sd_dir[s];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int32_t h = E.sd_hits[4 * s + k];
                pix[k] = lpt_px(E.px_x[h], E.px_y[h], E.px_z[h]);
            }
            link_scan<KIND, WPS>(E, K, P, s, ev, d, pix, q, n_acc, sm, w, 0u, false);
        }
        if (l == 0) sm.cnt[w] = n_acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int k = 0; k < PX_LW; ++k) tot += sm.cnt[k];
            sm.base = tot ? atomicAdd(&E.gc[KIND == 5 ? GC_PX5 : GC_PX3], tot) : 0u;
        }
        __syncthreads();
        // the waves of one seed are adjacent, so each seed's range is consecutive
        uint32_t mine = sm.base;
        for (int k = 0; k < w; ++k) mine += sm.cnt[k];
        if (act) {
            const uint32_t cap = (uint32_t)E.cap_pxc;
            if (l == 0 && q == 0) {
                uint32_t all = 0;
                for (int k = 0; k < WPS; ++k) all += sm.cnt[w + k];
                const uint32_t first = mine < cap ? mine : cap;
                const uint32_t last = mine + all < cap ? mine + all : cap;
                sd_c[s] = make_int2((int)first, (int)(last - first));
                if (mine + all > cap) atomicOr(&E.gc[GC_OVERFLOW], 1u << OT_COUNT);
            }
            const uint32_t staged = n_acc < PX_STAGE ? n_acc : PX_STAGE;
            for (uint32_t k = l; k < staged; k += 64) {
                const uint32_t at = mine + k;
                if (at < cap) {
                    c_seed[at] = s;
                    c_obj[at] = sm.obj[w][k];
                    c_score[at] = sm.score[w][k];
                }
            }
            if (n_acc > PX_STAGE) {
                uint32_t again = 0;
                link_scan<KIND, WPS>(E, K, P, s, ev, d, pix, q, again, sm, w, mine, true);
            }
        }
        __syncthreads();   // the stage is rewritten by the next round
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


// every candidate's key (score bits, seed's index in its event) into the
// per-hit minima of its collection
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

// per-event hit index of outer hit j of an object
template <int KIND>
__device__ __forceinline__ int32_t c_orig(const EvDev &E, int32_t obj, int j)
{
    return hit_orig(E, c_ohit<KIND>(E, obj, j));
}

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_pxd_keep(EvDev E, int n_mod)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<KIND>(E);
    for (uint32_t c0 = blockIdx.x * BLOCK; c0 < n; c0 += gridDim.x * BLOCK) {
        const uint32_t c = c0 + threadIdx.x;
        if (c >= n) continue;
        const unsigned long long key = c_key<KIND>(E, c);
        const int32_t s = KIND == 5 ? E.c5_seed[c] : E.c3_seed[c];
        const int32_t o = KIND == 5 ? E.c5_obj[c] : E.c3_obj[c];
        bool keep = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) keep = keep && E.hmin_p[E.sd_hits[4 * s + k]] == key;
#pragma unroll
        for (int j = 0; j < 2 * KIND; ++j) keep = keep && E.hmin_o[c_ohit<KIND>(E, o, j)] == key;
        if (keep) {
            // equal (score, seed): the smaller outer hit tuple wins; the
            // seed's candidates are consecutive
            const float sc = KIND == 5 ? E.c5_score[c] : E.c3_score[c];
            const int2 rg = (KIND == 5 ? E.sd_c5 : E.sd_c3)[s];
            for (uint32_t u = (uint32_t)rg.x; u < (uint32_t)(rg.x + rg.y) && keep; ++u) {
                if (u == c) continue;
                const float scu = KIND == 5 ? E.c5_score[u] : E.c3_score[u];
                if (__float_as_uint(scu) != __float_as_uint(sc)) continue;
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
            if (keep) E.sd_used[s] = 1;
            (void)agg_add(pl(E, E.pl_cnt, PXL_D5), E.sd_ev[s] * PX_NB + dir_bin(E.sd_dir[s]), keep);
        } else {
            E.c3_keep[c] = keep;
        }
    }
    (void)n_mod;
}

// ---------------------------------------------------------------- cross-cleaning
// any direction of the event's list within dr2 of d: the whole wave scans
// the list's azimuth bins around d (half-width wdr) 64 entries at a time
// (wave-uniform arguments)
__device__ __forceinline__ bool wave_near_any(const EvDev &E, int list, int ev, const float4 *dirs,
                                              const float4 &d, float dr2, float wdr)
{
    const int32_t *off = pl(E, E.pl_off, list);
    int a[2], b[2];
    window_bins(d, wdr, a[0], b[0], a[1], b[1]);
    for (int part = 0; part < 2; ++part) {
        if (a[part] > b[part]) continue;
        const int32_t i0 = off[ev * PX_NB + a[part]], i1 = off[ev * PX_NB + b[part] + 1];
        for (int32_t bb = i0; bb < i1; bb += 64) {
            const int32_t i = bb + px_lane();
            if (__ballot(i < i1 && close_dir(d, dirs[i], dr2))) return true;
        }
    }
    return false;
}

// the run of objects [first, last) of the wave in a one-wave-per-object pass
__device__ __forceinline__ void wave_run(uint32_t n, uint32_t &first, uint32_t &last, uint32_t &step)
{
    const uint32_t w = blockIdx.x * WAVES + (threadIdx.x >> 6);
    first = w * PX_WCHUNK;
    step = gridDim.x * WAVES * PX_WCHUNK;
    last = first + PX_WCHUNK < n ? first + PX_WCHUNK : n;
}

// surviving pT5: their directions into the event list, their hits flagged
__global__ __launch_bounds__(BLOCK) void k_pt5_mark(EvDev E)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<5>(E);
    const int32_t *off = pl(E, E.pl_off, PXL_D5);
    int32_t *fill = pl(E, E.pl_fill, PXL_D5);
    for (uint32_t c0 = blockIdx.x * BLOCK; c0 < n; c0 += gridDim.x * BLOCK) {
        const uint32_t c = c0 + threadIdx.x;
        const bool act = c < n && E.c5_keep[c];
        int32_t s = 0;
        int ev = 0;
        if (act) {
            s = E.c5_seed[c];
            ev = E.sd_ev[s] * PX_NB + dir_bin(E.sd_dir[s]);
        }
        const int32_t at = agg_add(fill, ev, act);
        if (!act) continue;
        const int32_t o = E.c5_obj[c];
        E.pl_d5[off[ev] + at] = E.sd_dir[s];
        for (int k = 0; k < 4; ++k) E.hflag_p[E.sd_hits[4 * s + k]] = 1;
        for (int j = 0; j < 10; ++j) E.hflag_o[c_ohit<5>(E, o, j)] = 1;
    }
    // the pT5 minima are read no more: reset for the pT3 duplicate removal
    rekey_body(E, true);
}

// pT3 near a pT5 or sharing a hit with one are duplicates (one wave per
// candidate: lane k < 4 reads pixel hit k's flag, lane 4 + j outer hit j's)
__global__ __launch_bounds__(BLOCK) void k_pt3_clean(EvDev E, PixConsts P)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<3>(E);
    const int l = px_lane();
    int32_t *cnt = pl(E, E.pl_cnt, PXL_D3);
    uint32_t first, last, step;
    wave_run(n, first, last, step);
    for (; first < n; first += step, last = first + PX_WCHUNK < n ? first + PX_WCHUNK : n) {
        EvRun run;
        for (uint32_t c = first; c < last; ++c) {
            if (!E.c3_keep[c]) continue;
            const int32_t s = E.c3_seed[c], o = E.c3_obj[c];
            bool hit = false;
            if (l < 4) hit = E.hflag_p[E.sd_hits[4 * s + l]] != 0;
            else if (l < 10) hit = E.hflag_o[c_ohit<3>(E, o, l - 4)] != 0;
            const int ev = E.sd_ev[s];
            const float4 d = E.sd_dir[s];
            bool keep = __ballot(hit) == 0ull;
            if (keep) keep = !wave_near_any(E, PXL_D5, ev, E.pl_d5, d, P.dr2, P.wdr);
            if (l == 0) E.c3_keep[c] = keep;
            if (keep) run.add(cnt, ev * PX_NB + dir_bin(d));
        }
        run.flush(cnt);
    }
}

// cleaned pT3: directions into the event list, hits flagged, seeds used
__global__ __launch_bounds__(BLOCK) void k_pt3_mark(EvDev E)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = n_cand<3>(E);
    const int32_t *off = pl(E, E.pl_off, PXL_D3);
    int32_t *fill = pl(E, E.pl_fill, PXL_D3);
    for (uint32_t c0 = blockIdx.x * BLOCK; c0 < n; c0 += gridDim.x * BLOCK) {
        const uint32_t c = c0 + threadIdx.x;
        const bool act = c < n && E.c3_keep[c];
        int32_t s = 0;
        int ev = 0;
        if (act) {
            s = E.c3_seed[c];
            ev = E.sd_ev[s] * PX_NB + dir_bin(E.sd_dir[s]);
        }
        const int32_t at = agg_add(fill, ev, act);
        if (!act) continue;
        const int32_t o = E.c3_obj[c];
        E.pl_d3[off[ev] + at] = E.sd_dir[s];
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
    const int l = px_lane();
    int32_t *cnt = pl(E, E.pl_cnt, PXL_DT);
    uint32_t first, last, step;
    wave_run(n5, first, last, step);
    for (; first < n5; first += step, last = first + PX_WCHUNK < n5 ? first + PX_WCHUNK : n5) {
        EvRun run;
        for (uint32_t v = first; v < last; ++v) {
            const int32_t t = obj_at(E, OT_T5, s_pre, v);
            bool keep = E.t5_keep[t] != 0;
            if (keep) {
                const bool hit = l < 10 && E.hflag_o[c_ohit<5>(E, t, l)] != 0;
                keep = __ballot(hit) == 0ull;
                const int ev = md_event(E, E.t5_md0[t], n_mod);
                const float4 d = E.t5_dir[t];
                if (keep) keep = !wave_near_any(E, PXL_D5, ev, E.pl_d5, d, P.dr2, P.wdr);
                if (keep) keep = !wave_near_any(E, PXL_D3, ev, E.pl_d3, d, P.dr2, P.wdr);
                if (keep) run.add(cnt, ev * PX_NB + dir_bin(d));
            }
            if (l == 0) E.t5_clean[t] = keep;
        }
        run.flush(cnt);
    }
}

__global__ __launch_bounds__(BLOCK) void k_t5_clean_fill(EvDev E, int n_mod)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n5 = obj_prefix(E, OT_T5, s_pre);
    const int32_t *off = pl(E, E.pl_off, PXL_DT);
    int32_t *fill = pl(E, E.pl_fill, PXL_DT);
    for (uint32_t v0 = blockIdx.x * BLOCK; v0 < n5; v0 += gridDim.x * BLOCK) {
        const uint32_t v = v0 + threadIdx.x;
        int32_t t = 0;
        int ev = 0;
        bool act = false;
        if (v < n5) {
            t = obj_at(E, OT_T5, s_pre, v);
            act = E.t5_clean[t] != 0;
            if (act) ev = md_event(E, E.t5_md0[t], n_mod) * PX_NB + dir_bin(E.t5_dir[t]);
        }
        const int32_t at = agg_add(fill, ev, act);
        if (act) E.pl_dt[off[ev] + at] = E.t5_dir[t];
    }
    // the pT3 minima are read no more: reset for the pLS cleaning
    rekey_body(E, false);
}

// unlinked pLS: a pixel hit held by a candidate, or near one, is a
// duplicate; the rest mark their pixel hits with their index (minimum)
__global__ __launch_bounds__(BLOCK) void k_pls_clean(EvDev E, PixConsts P)
{
    if (upstream_overflow(E)) return;
    const uint32_t n_sd = (uint32_t)E.desc[D_NSEEDS];
    const int l = px_lane();
    uint32_t first, last, step;
    wave_run(n_sd, first, last, step);
    for (; first < n_sd; first += step, last = first + PX_WCHUNK < n_sd ? first + PX_WCHUNK : n_sd) {
        for (uint32_t s = first; s < last; ++s) {
            if (E.sd_used[s]) continue;
            const bool hit = l < 4 && E.hflag_p[E.sd_hits[4 * s + l]] != 0;
            bool keep = __ballot(hit) == 0ull;
            const int ev = E.sd_ev[s];
            const float4 d = E.sd_dir[s];
            if (keep) keep = !wave_near_any(E, PXL_D5, ev, E.pl_d5, d, P.dr2, P.wdr);
            if (keep) keep = !wave_near_any(E, PXL_D3, ev, E.pl_d3, d, P.dr2, P.wdr);
            if (keep) keep = !wave_near_any(E, PXL_DT, ev, E.pl_dt, d, P.dr2, P.wdr);
            if (l == 0) E.sd_keep[s] = keep;
            if (keep && l < 4)
                atomicMin(&E.hmin_p[E.sd_hits[4 * s + l]], (unsigned long long)(uint32_t)E.sd_local[s]);
        }
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
    // waves per seed in the link scans: a pT5 window holds a few dozen kept
    // quintuplets, a pT3 window hundreds of triplets
    constexpr int PX_WPS5 = 1, PX_WPS3 = 4;
    const int g_link5 = px_grid(E.cap_seeds, PX_LW / PX_WPS5);
    const int g_link3 = px_grid(E.cap_seeds, PX_LW / PX_WPS3);
    const int g_c = px_grid(E.cap_pxc, BLOCK);
    const int g_obj = px_grid((int64_t)E.rc[OT_T3] * NSH, BLOCK);
    // one wave per object, PX_WCHUNK objects per wave
    const int g_cw = px_grid(E.cap_pxc, WAVES * PX_WCHUNK);
    const int g_objw = px_grid((int64_t)E.rc[OT_T5] * NSH, WAVES * PX_WCHUNK);
    const int g_sdc = px_grid(E.cap_seeds, WAVES * PX_WCHUNK);
    hipLaunchKernelGGL(k_px_init, dim3(g_hits), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_obj_dir, dim3(g_obj), dim3(BLOCK), 0, s, E, n_mod);
    hipLaunchKernelGGL(k_pl_scan, dim3(2), dim3(1024), 0, s, E, (int)PXL_K5, (int)PXL_K3, PX_NB);
    hipLaunchKernelGGL(k_obj_fill, dim3(g_obj), dim3(BLOCK), 0, s, E, n_mod);
    // pT5
    hipLaunchKernelGGL((k_px_link<5, PX_WPS5>), dim3(g_link5), dim3(PX_LW * 64), 0, s, E, K, P);
    hipLaunchKernelGGL(k_pxd_min<5>, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_pxd_keep<5>, dim3(g_c), dim3(BLOCK), 0, s, E, n_mod);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_D5, (int)PXL_D5, PX_NB);
    hipLaunchKernelGGL(k_pt5_mark, dim3(std::max(g_c, g_hits)), dim3(BLOCK), 0, s, E);
    // pT3 from the seeds no pT5 uses
    hipLaunchKernelGGL((k_px_link<3, PX_WPS3>), dim3(g_link3), dim3(PX_LW * 64), 0, s, E, K, P);
    hipLaunchKernelGGL(k_pxd_min<3>, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_pxd_keep<3>, dim3(g_c), dim3(BLOCK), 0, s, E, n_mod);
    // cross-cleaning
    hipLaunchKernelGGL(k_pt3_clean, dim3(g_cw), dim3(BLOCK), 0, s, E, P);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_D3, (int)PXL_D3, PX_NB);
    hipLaunchKernelGGL(k_pt3_mark, dim3(g_c), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_t5_clean, dim3(g_objw), dim3(BLOCK), 0, s, E, P, n_mod);
    hipLaunchKernelGGL(k_pl_scan, dim3(1), dim3(1024), 0, s, E, (int)PXL_DT, (int)PXL_DT, PX_NB);
    hipLaunchKernelGGL(k_t5_clean_fill, dim3(std::max(g_obj, g_hits)), dim3(BLOCK), 0, s, E, n_mod);
    hipLaunchKernelGGL(k_pls_clean, dim3(g_sdc), dim3(BLOCK), 0, s, E, P);
    hipLaunchKernelGGL(k_pls_keep, dim3(g_sd), dim3(BLOCK), 0, s, E);
    return hipGetLastError();
}

}  // namespace lst
