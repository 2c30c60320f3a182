// Stage kernels of the Segment Linking chain for gfx950 (wave64).
//
// Structure shared by the object stages: one wavefront owns one "slot"
// (event x module) and enumerates the slot's candidate combinations 64 at a
// time, one per lane.  Candidate lists that are concatenations of several
// groups (map edges, outgoing segments, outgoing triplets) are flattened with
// a wave-wide inclusive scan of the group sizes; a lane finds its group by a
// binary search over that scan held in registers (cross-lane reads, no LDS).
// Accepted objects are compacted with ballot + popcount, no per-object
// atomics: pass 1 counts, the block reserves its whole range with ONE atomic,
// pass 2 recomputes the (cheap) predicate and writes each object at its
// slot-contiguous position.  The output of a stage stays grouped by its inner
// object, which is exactly the index the next stage needs.
#include "lst_cuts.hpp"

namespace lst {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ unsigned long long lanes_below()
{
    return (1ull << lane_id()) - 1ull;
}

// inclusive scan over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (l >= d) v += t;
    }
    return v;
}

// smallest lane e with incl[e] > j (incl non-decreasing, j < incl[63])
__device__ __forceinline__ int wave_find(uint32_t incl, uint32_t j)
{
    int lo = 0, hi = 63;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        int mid = (lo + hi) >> 1;
        uint32_t v = __shfl(incl, mid, 64);
        if (v > j) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Block-wide reservation: every thread of the block must call it.  Returns
// the first output index of the calling wave; `ovf` is set for every wave of
// the block when the block's range does not fit the capacity.
__device__ __forceinline__ uint32_t block_reserve(uint32_t wave_total, int32_t *counter,
                                                  int64_t cap, int32_t *gc, int stage_bit,
                                                  bool &ovf)
{
    __shared__ uint32_t s_cnt[WAVES];
    __shared__ uint32_t s_base;
    __shared__ int s_ovf;
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) s_cnt[w] = wave_total;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int i = 0; i < WAVES; ++i) tot += s_cnt[i];
        uint32_t base = tot ? atomicAdd((uint32_t *)counter, tot) : 0u;
        int o = ((uint64_t)base + tot) > (uint64_t)cap;
        if (o) atomicOr(&gc[GC_OVERFLOW], 1 << stage_bit);
        s_base = base;
        s_ovf = o;
    }
    __syncthreads();
    uint32_t off = s_base;
    for (int i = 0; i < w; ++i) off += s_cnt[i];
    ovf = s_ovf != 0;
    __syncthreads();
    return off;
}

// ---------------------------------------------------------------- zero fill
__global__ void k_zero(uint4 *p, size_t n16)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_zero(const EvDev &, void *zero_base, size_t zero_bytes, hipStream_t s)
{
    size_t n16 = zero_bytes / 16;
    int blocks = (int)((n16 + BLOCK - 1) / BLOCK);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(BLOCK), 0, s, (uint4 *)zero_base, n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------- a0: sort
__device__ __forceinline__ int event_of(const int32_t *off, int n_ev, int32_t h)
{
    int lo = 0, hi = n_ev - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= h) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int hit_key(const EvDev &E, int n_mod, int32_t h, int &ev)
{
    ev = event_of(E.hit_off, E.n_ev, h);
    int32_t m = E.module[h];
    uint8_t s = E.sensor[h];
    if (m < 0 || m >= n_mod || s > 1) return -1;
    return 2 * (ev * n_mod + m) + s;
}

__global__ void k_hist(EvDev E, int n_mod)
{
    int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= E.n_hits) return;
    int ev;
    int key = hit_key(E, n_mod, h, ev);
    if (key < 0) {
        atomicOr(&E.gc[GC_ERROR], 1);
        return;
    }
    atomicAdd(&E.bcnt[key], 1u);
}

// exclusive scan of bcnt[0..n) into boff[0..n], three phases over tiles of 1024
constexpr int SCAN_TILE = 1024;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &total)
{
    __shared__ uint32_t s_w[WAVES];
    uint32_t incl = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) s_w[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int i = 0; i < WAVES; ++i) {
        if (i < w) before += s_w[i];
        total += s_w[i];
    }
    __syncthreads();
    return before + incl - v;
}

__global__ void k_scan_reduce(const uint32_t *in, int n, uint32_t *bsum)
{
    int base = blockIdx.x * SCAN_TILE + threadIdx.x * 4;
    uint32_t v = 0;
    for (int k = 0; k < 4; ++k)
        if (base + k < n) v += in[base + k];
    uint32_t tot;
    block_excl_scan(v, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_top(uint32_t *bsum, int nb)
{
    // single block: exclusive scan of nb partials, nb <= 16 * BLOCK
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += BLOCK) {
        int i = b0 + threadIdx.x;
        uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

__global__ void k_scan_down(const uint32_t *in, int n, const uint32_t *bsum, uint32_t *out,
                            int32_t *gc)
{
    int base = blockIdx.x * SCAN_TILE + threadIdx.x * 4;
    uint32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, tot) + bsum[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == BLOCK - 1) {
        out[n] = ex;
        gc[GC_N_SORTED] = (int32_t)ex;
    }
}

__global__ void k_scatter(EvDev E, int n_mod)
{
    int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= E.n_hits) return;
    int ev;
    int key = hit_key(E, n_mod, h, ev);
    if (key < 0) return;
    // positions are taken from the top of the bin down; bcnt ends at zero
    uint32_t pos = E.boff[key] + atomicSub(&E.bcnt[key], 1u) - 1u;
    E.sx[pos] = E.x[h];
    E.sy[pos] = E.y[h];
    E.sz[pos] = E.z[h];
    E.sorig[pos] = h - E.hit_off[ev];
    E.hmin[pos] = 0xffffffffu;
    E.htie[pos] = 0;
}

hipError_t launch_sort(const EvDev &E, const ModDev &M, hipStream_t s)
{
    if (E.n_hits > 0) {
        int blocks = (E.n_hits + BLOCK - 1) / BLOCK;
        hipLaunchKernelGGL(k_hist, dim3(blocks), dim3(BLOCK), 0, s, E, M.n_mod);
    }
    int n = E.n_keys;
    int nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(BLOCK), 0, s, E.bcnt, n, E.bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, s, E.bsum, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(BLOCK), 0, s, E.bcnt, n, E.bsum, E.boff,
                       E.gc);
    if (E.n_hits > 0) {
        int blocks = (E.n_hits + BLOCK - 1) / BLOCK;
        hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(BLOCK), 0, s, E, M.n_mod);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- a1: MD
__device__ __forceinline__ ModF load_mod(const ModDev &M, int m)
{
    ModF f;
    f.cx = M.cx[m]; f.cy = M.cy[m]; f.cz = M.cz[m];
    f.ux = M.ux[m]; f.uy = M.uy[m]; f.uz = M.uz[m];
    f.vx = M.vx[m]; f.vy = M.vy[m]; f.vz = M.vz[m];
    f.g = M.g[m]; f.rl = M.rl[m];
    f.barrel = M.barrel[m];
    return f;
}

__global__ __launch_bounds__(BLOCK) void k_md(EvDev E, ModDev M, Consts K)
{
    const int lane = lane_id();
    const int slot = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const bool act = slot < E.n_slots;
    uint32_t lo0 = 0, up0 = 0, nlo = 0, nup = 0;
    if (act) {
        lo0 = E.boff[2 * slot];
        up0 = E.boff[2 * slot + 1];
        nlo = up0 - lo0;
        nup = E.boff[2 * slot + 2] - up0;
    }
    const uint32_t np = nlo * nup;
    const int m = act ? slot % M.n_mod : 0;
    ModF mod;
    if (np) mod = load_mod(M, m);
    uint32_t cnt = 0;
    for (uint32_t b = 0; b < np; b += 64) {
        uint32_t p = b + lane;
        bool ok = false;
        if (p < np) {
            uint32_t il = p / nup, iu = p - il * nup;
            uint32_t hl = lo0 + il, hu = up0 + iu;
            MdOut o;
            ok = md_accept(K, mod, E.sx[hl], E.sy[hl], E.sz[hl], E.sx[hu], E.sy[hu], E.sz[hu], o);
        }
        cnt += (uint32_t)__popcll(__ballot(ok));
    }
    bool ovf;
    uint32_t off = block_reserve(cnt, &E.gc[GC_MD], E.cap_md, E.gc, 0, ovf);
    if (!act) return;
    if (lane == 0) {
        E.md_start[slot] = (int32_t)off;
        E.md_cnt[slot] = ovf ? 0 : (int32_t)cnt;
    }
    if (ovf || cnt == 0) return;
    uint32_t pos = off;
    for (uint32_t b = 0; b < np; b += 64) {
        uint32_t p = b + lane;
        bool ok = false;
        uint32_t hl = 0, hu = 0;
        MdOut o;
        if (p < np) {
            uint32_t il = p / nup, iu = p - il * nup;
            hl = lo0 + il;
            hu = up0 + iu;
            ok = md_accept(K, mod, E.sx[hl], E.sy[hl], E.sz[hl], E.sx[hu], E.sy[hu], E.sz[hu], o);
        }
        unsigned long long mask = __ballot(ok);
        if (ok) {
            uint32_t i = pos + (uint32_t)__popcll(mask & lanes_below());
            float xL = E.sx[hl], yL = E.sy[hl];
            E.md_hlo[i] = (int32_t)hl;
            E.md_hup[i] = (int32_t)hu;
            E.md_slot[i] = slot;
            E.md_x[i] = xL;
            E.md_y[i] = yL;
            E.md_z[i] = E.sz[hl];
            E.md_r[i] = o.r;
            E.md_a[i] = o.a;
            E.md_ca[i] = o.ca;
            float dx = E.sx[hu] - xL, dy = E.sy[hu] - yL;
            E.md_dx[i] = dx;
            E.md_dy[i] = dy;
            E.md_dn[i] = sqrtf((dx * dx) + (dy * dy));
            E.md_bend[i] = o.bend;
            E.md_sv[i] = o.sv;
            E.md_bar[i] = (uint8_t)mod.barrel;
        }
        pos += (uint32_t)__popcll(mask);
    }
}

hipError_t launch_md(const EvDev &E, const ModDev &M, const Consts &K, hipStream_t s)
{
    int blocks = (E.n_slots + WAVES - 1) / WAVES;
    hipLaunchKernelGGL(k_md, dim3(blocks), dim3(BLOCK), 0, s, E, M, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- a2: segments
// Outer candidates of an inner MD: the MDs of every map edge of its module,
// in edge order.  Pass 1 counts, pass 2 writes.
template <bool WRITE>
__device__ __forceinline__ uint32_t seg_slot(const EvDev &E, const ModDev &M, const Consts &K,
                                             int slot, uint32_t pos, unsigned long long *cand)
{
    const int lane = lane_id();
    const int32_t sA = E.md_start[slot];
    const int32_t nA = E.md_cnt[slot];
    const int ev = slot / M.n_mod;
    const int m = slot - ev * M.n_mod;
    const int32_t e0 = M.map_ptr[m];
    const int32_t ne = M.map_ptr[m + 1] - e0;
    const int base_slot = ev * M.n_mod;
    uint32_t cnt = 0;
    for (int32_t ii = 0; ii < nA; ++ii) {
        const int32_t i = sA + ii;
        const MdV I = load_md(E, i);
        const uint32_t pos_i = pos + cnt;
        for (int32_t ec = 0; ec < ne; ec += 64) {
            int32_t e = ec + lane;
            uint32_t bc = 0;
            int32_t bs = 0;
            if (e < ne) {
                int b = base_slot + M.map_col[e0 + e];
                bs = E.md_start[b];
                bc = (uint32_t)E.md_cnt[b];
            }
            uint32_t incl = wave_incl_scan(bc);
            uint32_t tot = __shfl(incl, 63, 64);
            if (!WRITE && ii == 0) *cand += tot;
            for (uint32_t jc = 0; jc < tot; jc += 64) {
                uint32_t j = jc + lane;
                bool ok = false;
                int32_t o = 0;
                int src = wave_find(incl, j < tot ? j : tot - 1);
                uint32_t ex = __shfl(incl, src, 64) - __shfl(bc, src, 64);
                int32_t obs = __shfl(bs, src, 64);
                if (j < tot) {
                    o = obs + (int32_t)(j - ex);
                    const MdV O = load_md(E, o);
                    ok = seg_accept(K, I, O);
                }
                unsigned long long mask = __ballot(ok);
                if (WRITE && ok) {
                    uint32_t at = pos + cnt + (uint32_t)__popcll(mask & lanes_below());
                    E.seg_in[at] = i;
                    E.seg_out[at] = o;
                }
                cnt += (uint32_t)__popcll(mask);
            }
        }
        if (WRITE && lane == 0) {
            E.seg_start[i] = (int32_t)pos_i;
            E.seg_cnt[i] = (int32_t)(pos + cnt - pos_i);
        }
    }
    if (!WRITE && cand) *cand *= (unsigned long long)nA;
    return cnt;
}

__global__ __launch_bounds__(BLOCK) void k_seg(EvDev E, ModDev M, Consts K)
{
    const int slot = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const bool act = slot < E.n_slots;
    unsigned long long cand = 0;
    uint32_t cnt = act ? seg_slot<false>(E, M, K, slot, 0, &cand) : 0u;
    (void)cand;
    bool ovf;
    uint32_t off = block_reserve(cnt, &E.gc[GC_SEG], E.cap_seg, E.gc, 1, ovf);
    if (!act) return;
    if (ovf) {
        const int32_t sA = E.md_start[slot], nA = E.md_cnt[slot];
        for (int32_t ii = lane_id(); ii < nA; ii += 64) {
            E.seg_start[sA + ii] = 0;
            E.seg_cnt[sA + ii] = 0;
        }
        return;
    }
    seg_slot<true>(E, M, K, slot, off, nullptr);
}

hipError_t launch_seg(const EvDev &E, const ModDev &M, const Consts &K, hipStream_t s)
{
    int blocks = (E.n_slots + WAVES - 1) / WAVES;
    hipLaunchKernelGGL(k_seg, dim3(blocks), dim3(BLOCK), 0, s, E, M, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- a3: triplets
template <bool WRITE>
__device__ __forceinline__ uint32_t t3_slot(const EvDev &E, const Consts &K, int slot,
                                            uint32_t pos, unsigned long long *cand)
{
    const int lane = lane_id();
    const int32_t sA = E.md_start[slot];
    const int32_t nA = E.md_cnt[slot];
    uint32_t cnt = 0;
    for (int32_t ii = 0; ii < nA; ++ii) {
        const int32_t a = sA + ii;
        const int32_t ns1 = E.seg_cnt[a];
        const int32_t s10 = E.seg_start[a];
        const uint32_t pos_a = pos + cnt;
        if (ns1 > 0) {
            const MdV A = load_md(E, a);
            for (int32_t c1 = 0; c1 < ns1; c1 += 64) {
                int32_t k = c1 + lane;
                int32_t b = 0, bs = 0;
                uint32_t nb = 0;
                if (k < ns1) {
                    b = E.seg_out[s10 + k];
                    bs = E.seg_start[b];
                    nb = (uint32_t)E.seg_cnt[b];
                }
                uint32_t incl = wave_incl_scan(nb);
                uint32_t tot = __shfl(incl, 63, 64);
                if (!WRITE) *cand += tot;
                for (uint32_t jc = 0; jc < tot; jc += 64) {
                    uint32_t j = jc + lane;
                    int src = wave_find(incl, j < tot ? j : tot - 1);
                    uint32_t ex = __shfl(incl, src, 64) - __shfl(nb, src, 64);
                    int32_t bb = __shfl(b, src, 64);
                    int32_t bbs = __shfl(bs, src, 64);
                    bool ok = false;
                    int32_t c = 0;
                    float kk = 0.0f;
                    if (j < tot) {
                        c = E.seg_out[bbs + (int32_t)(j - ex)];
                        const MdV B = load_md(E, bb);
                        const MdV C = load_md(E, c);
                        ok = t3_accept(K, A, B, C, kk);
                    }
                    unsigned long long mask = __ballot(ok);
                    if (WRITE && ok) {
                        uint32_t at = pos + cnt + (uint32_t)__popcll(mask & lanes_below());
                        E.t3_a[at] = a;
                        E.t3_b[at] = bb;
                        E.t3_c[at] = c;
                        E.t3_k[at] = kk;
                    }
                    cnt += (uint32_t)__popcll(mask);
                }
            }
        }
        if (WRITE && lane == 0) {
            E.t3_start[a] = (int32_t)pos_a;
            E.t3_cnt[a] = (int32_t)(pos + cnt - pos_a);
        }
    }
    return cnt;
}

__global__ __launch_bounds__(BLOCK) void k_t3(EvDev E, ModDev M, Consts K)
{
    const int slot = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const bool act = slot < E.n_slots;
    unsigned long long cand = 0;
    uint32_t cnt = act ? t3_slot<false>(E, K, slot, 0, &cand) : 0u;
    (void)cand;
    bool ovf;
    uint32_t off = block_reserve(cnt, &E.gc[GC_T3], E.cap_t3, E.gc, 2, ovf);
    if (!act) return;
    if (ovf) {
        const int32_t sA = E.md_start[slot], nA = E.md_cnt[slot];
        for (int32_t ii = lane_id(); ii < nA; ii += 64) {
            E.t3_start[sA + ii] = 0;
            E.t3_cnt[sA + ii] = 0;
        }
        return;
    }
    t3_slot<true>(E, K, slot, off, nullptr);
}

hipError_t launch_t3(const EvDev &E, const ModDev &M, const Consts &K, hipStream_t s)
{
    int blocks = (E.n_slots + WAVES - 1) / WAVES;
    hipLaunchKernelGGL(k_t3, dim3(blocks), dim3(BLOCK), 0, s, E, M, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- a4: quintuplets
template <bool WRITE>
__device__ __forceinline__ uint32_t t5_slot(const EvDev &E, const Consts &K, int slot,
                                            uint32_t pos, unsigned long long *cand)
{
    const int lane = lane_id();
    const int32_t sA = E.md_start[slot];
    const int32_t nA = E.md_cnt[slot];
    uint32_t cnt = 0;
    for (int32_t ii = 0; ii < nA; ++ii) {
        const int32_t a = sA + ii;
        const int32_t nt1 = E.t3_cnt[a];
        const int32_t t10 = E.t3_start[a];
        if (nt1 <= 0) continue;
        const MdV A = load_md(E, a);
        for (int32_t c1 = 0; c1 < nt1; c1 += 64) {
            int32_t k = c1 + lane;
            int32_t t1 = 0, cs = 0;
            uint32_t nc = 0;
            if (k < nt1) {
                t1 = t10 + k;
                int32_t c = E.t3_c[t1];
                cs = E.t3_start[c];
                nc = (uint32_t)E.t3_cnt[c];
            }
            uint32_t incl = wave_incl_scan(nc);
            uint32_t tot = __shfl(incl, 63, 64);
            if (!WRITE) *cand += tot;
            for (uint32_t jc = 0; jc < tot; jc += 64) {
                uint32_t j = jc + lane;
                int src = wave_find(incl, j < tot ? j : tot - 1);
                uint32_t ex = __shfl(incl, src, 64) - __shfl(nc, src, 64);
                int32_t tt1 = __shfl(t1, src, 64);
                int32_t tcs = __shfl(cs, src, 64);
                bool ok = false;
                int32_t b = 0, c = 0, d = 0, e = 0;
                float score = 0.0f;
                if (j < tot) {
                    int32_t t2 = tcs + (int32_t)(j - ex);
                    b = E.t3_b[tt1];
                    c = E.t3_c[tt1];
                    d = E.t3_b[t2];
                    e = E.t3_c[t2];
                    float kin = E.t3_k[tt1], kout = E.t3_k[t2];
                    const MdV B = load_md(E, b);
                    const MdV C = load_md(E, c);
                    const MdV D = load_md(E, d);
                    const MdV Ee = load_md(E, e);
                    ok = t5_accept(K, A, B, C, D, Ee, kin, kout, score);
                }
                unsigned long long mask = __ballot(ok);
                if (WRITE && ok) {
                    uint32_t at = pos + cnt + (uint32_t)__popcll(mask & lanes_below());
                    E.t5_md0[at] = a;
                    E.t5_md1[at] = b;
                    E.t5_md2[at] = c;
                    E.t5_md3[at] = d;
                    E.t5_md4[at] = e;
                    E.t5_score[at] = score;
                    E.t5_keep[at] = 0;
                }
                cnt += (uint32_t)__popcll(mask);
            }
        }
    }
    return cnt;
}

__global__ __launch_bounds__(BLOCK) void k_t5(EvDev E, ModDev M, Consts K)
{
    const int slot = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const bool act = slot < E.n_slots;
    unsigned long long cand = 0;
    uint32_t cnt = act ? t5_slot<false>(E, K, slot, 0, &cand) : 0u;
    (void)cand;
    bool ovf;
    uint32_t off = block_reserve(cnt, &E.gc[GC_T5], E.cap_t5, E.gc, 3, ovf);
    if (!act) return;
    if (ovf) return;
    t5_slot<true>(E, K, slot, off, nullptr);
}

hipError_t launch_t5(const EvDev &E, const ModDev &M, const Consts &K, hipStream_t s)
{
    int blocks = (E.n_slots + WAVES - 1) / WAVES;
    hipLaunchKernelGGL(k_t5, dim3(blocks), dim3(BLOCK), 0, s, E, M, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- a5: dedup
// A quintuplet survives iff for each of its hits it has the smallest key
// (score, hit tuple) among the quintuplets using that hit.  Scores are
// non-negative, so their bit patterns order like the floats.
__device__ __forceinline__ int t5_md(const EvDev &E, int32_t t, int j)
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
    int32_t md = t5_md(E, t, j >> 1);
    return (j & 1) ? E.md_hup[md] : E.md_hlo[md];
}

__device__ __forceinline__ int32_t n_t5(const EvDev &E)
{
    int64_t n = E.gc[GC_T5];
    if (E.gc[GC_OVERFLOW] & 8) n = 0;
    return (int32_t)(n < E.cap_t5 ? n : E.cap_t5);
}

__global__ void k_dedup_min(EvDev E)
{
    const int32_t n = n_t5(E);
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        uint32_t key = __float_as_uint(E.t5_score[t]);
        for (int j = 0; j < 10; ++j) atomicMin(&E.hmin[t5_hit(E, t, j)], key);
    }
}

// Quintuplets reaching a hit's minimum score are recorded in TIE_SLOTS
// per-hit slots; exact score ties are common (two quintuplets that differ
// only in the upper hit of one mini-doublet have the same anchors, hence the
// same score) and are resolved by the hit tuple.
__global__ void k_dedup_tie(EvDev E)
{
    const int32_t n = n_t5(E);
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        uint32_t key = __float_as_uint(E.t5_score[t]);
        for (int j = 0; j < 10; ++j) {
            int32_t h = t5_hit(E, t, j);
            if (E.hmin[h] == key) {
                int k = atomicAdd(&E.htie[h], 1);
                if (k < TIE_SLOTS) E.hslot[(size_t)h * TIE_SLOTS + k] = t;
            }
        }
    }
}

// lexicographic order of the (per-event) hit-index tuples
__device__ __forceinline__ bool tuple_less(const EvDev &E, int32_t u, int32_t t)
{
    for (int j = 0; j < 10; ++j) {
        int32_t a = E.sorig[t5_hit(E, u, j)], b = E.sorig[t5_hit(E, t, j)];
        if (a != b) return a < b;
    }
    return false;
}

__global__ void k_dedup_keep(EvDev E)
{
    const int32_t n = n_t5(E);
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const float sc = E.t5_score[t];
        const uint32_t key = __float_as_uint(sc);
        bool keep = true;
        for (int j = 0; j < 10 && keep; ++j) {
            int32_t h = t5_hit(E, t, j);
            if (E.hmin[h] != key) { keep = false; break; }
            const int nt = E.htie[h];
            if (nt <= 1) continue;
            if (nt <= TIE_SLOTS) {
                for (int k = 0; k < nt && keep; ++k) {
                    int32_t u = E.hslot[(size_t)h * TIE_SLOTS + k];
                    if (u != t && tuple_less(E, u, t)) keep = false;
                }
            } else {
                // more ties than slots: scan every quintuplet (never seen in practice)
                for (int32_t u = 0; u < n && keep; ++u) {
                    if (u == t || E.t5_score[u] != sc) continue;
                    bool uses = false;
                    for (int k = 0; k < 10; ++k) uses |= (t5_hit(E, u, k) == h);
                    if (uses && tuple_less(E, u, t)) keep = false;
                }
            }
        }
        E.t5_keep[t] = keep ? 1 : 0;
    }
}

hipError_t launch_dedup(const EvDev &E, const ModDev &M, hipStream_t s)
{
    int blocks = 1024;
    hipLaunchKernelGGL(k_dedup_min, dim3(blocks), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_dedup_tie, dim3(blocks), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_dedup_keep, dim3(blocks), dim3(BLOCK), 0, s, E);
    return hipGetLastError();
}

}  // namespace lst
