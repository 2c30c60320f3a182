// Stage kernels of the Segment Linking chain for gfx950 (wave64).
//
// Work decomposition of the object stages: a wavefront takes P inner
// objects per round (module slots for mini-doublets, inner mini-doublets for
// segments, triplets and quintuplets; a group of G = 64 / P lanes, or one
// lane, sets each up) and walks all their candidate combinations as one
// list, 64 at a time, one per lane.  Candidate lists that are
// concatenations of several ranges (map edges, outgoing segments, outgoing
// triplets) are flattened with a wave-wide inclusive scan of the range
// sizes, and a lane finds its range from that scan with cross-lane reads.
// Accepted objects are compacted with ballot + popcount into an LDS staging
// buffer; the wave then reserves its output range with one atomic on one of
// the shard counters of its XCD sector and copies its staged objects out.
// Kernels are grid-stride over the inner objects, whose number is only
// known on the device.  When the grid covers a sector in one pass the
// sector's inner objects are spread over the waves (heavy modules do not
// pile up in one wave); otherwise consecutive objects go together, and on
// batches the segment stage enumerates the candidates of a run of MDs of
// one module once.
//
// Why not one global counter: device-scope atomics on one address are
// serialised across the chip (measured ~0.1 us apiece through 16 counters),
// so per-object or per-wave atomics on a shared counter cost more than the
// whole stage.
#include "lst_access.hpp"
#include "lst_cuts.hpp"

namespace lst {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ unsigned long long lanes_below()
{
    return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ void wave_lds_sync()
{
    // orders the wave's LDS writes before its later LDS reads by other lanes
    // (a wave's LDS operations complete in issue order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive max-scan of non-negative values over the 64 lanes: shifts within
// rows of 16 lanes, then the last lane of a row broadcast to the next rows
// (DPP row_shr:1,2,4,8, row_bcast:15, row_bcast:31)
__device__ __forceinline__ int wave_max_scan(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
    return v;
}

// Lane l owns c consecutive positions of a list, ending at its inclusive
// prefix incl.  Returns the owner of position jc + lane (positions past the
// end map to the last owner): each owner marks where its range enters the
// window [jc, jc + 64) in the wave's LDS row `mark`, and a max-scan fills
// the gaps.
__device__ __forceinline__ int chunk_src(uint32_t incl, uint32_t c, uint32_t jc, int *mark)
{
    const int l = lane_id();
    mark[l] = 0;
    wave_lds_sync();
    const uint32_t ex = incl - c;
    if (c > 0) {
        if (ex >= jc && ex < jc + 64u) mark[ex - jc] = l + 1;
        else if (ex < jc && incl > jc) mark[0] = l + 1;
    }
    wave_lds_sync();
    const int v = mark[l];
    wave_lds_sync();
    return wave_max_scan(v) - 1;
}

// inclusive scan over the 64 lanes of a wave (the same DPP pattern as
// wave_max_scan, adding; lanes outside a shift or a broadcast add zero)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
    return (uint32_t)x;
}

// smallest lane e with incl[e] > j (incl non-decreasing, j < incl[63]);
// every lane of the wave must take part
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

// A wave split into P = 64 / G groups of G lanes: each group sets up its
// own inner object, so P objects' loads are in flight per wave; Grp<64>
// gives the whole-wave scan, broadcast and search the stages use to walk
// their candidates as one list.
template <int G>
struct Grp {
    static constexpr int P = 64 / G;
    int lane, g;
    __device__ __forceinline__ Grp() : lane(threadIdx.x & (G - 1)), g((threadIdx.x & 63) / G) {}
    template <class T>
    __device__ __forceinline__ T bcast(T v, int src) const { return __shfl(v, src, G); }
    // exclusive prefix of a per-group value over the wave's groups, and the sum
    __device__ __forceinline__ uint32_t wave_prefix(uint32_t v, uint32_t &sum) const
    {
        uint32_t ex = 0;
        sum = 0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const uint32_t c = __shfl(v, q * G, 64);
            if (q < g) ex += c;
            sum += c;
        }
        return ex;
    }
};

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t t = __shfl_xor(v, d, 64);
        v = t > v ? t : v;
    }
    return v;
}

// ---------------------------------------------------------------- regions
// Objects of one type live in NSH regions; n_s = min(counter_s, rc) of them
// in region s.  A wave maps a compact index v to its array index with a scan
// of the region sizes held in the first lanes.
// The regions written by the blocks of XCD sector x (shards x, x + NXCD, ...),
// as a compact index: the object stages read their inner objects from the
// sector their own blocks belong to.
struct XRegions {
    uint32_t incl, size, total, rc;
    int x;
};

__device__ __forceinline__ XRegions load_regions_x(const EvDev &E, int type, int x)
{
    XRegions R;
    R.x = x;
    R.rc = E.rc[type];
    uint32_t n = 0;
    if (lane_id() < NSH / NXCD) {
        const uint32_t c = E.gc[gc_shard(type, x + NXCD * lane_id())];
        n = c < R.rc ? c : R.rc;
    }
    R.size = n;
    R.incl = wave_incl_scan(n);
    R.total = __shfl(R.incl, 63, 64);
    return R;
}

// v < R.total (may differ between lanes); every lane of the wave takes part
__device__ __forceinline__ int32_t region_index_x(const XRegions &R, uint32_t v)
{
    const int r = wave_find(R.incl, v);
    const uint32_t ex = __shfl(R.incl, r, 64) - __shfl(R.size, r, 64);
    return (int32_t)((uint32_t)(R.x + NXCD * r) * R.rc + (v - ex));
}

// this block's sector, its rank among the sector's blocks and their number
struct XBlock {
    int x;
    uint32_t rank, count;
};

__device__ __forceinline__ XBlock xcd_block()
{
    XBlock b;
    b.x = (int)(blockIdx.x % NXCD);
    b.rank = blockIdx.x / NXCD;
    b.count = (gridDim.x - (uint32_t)b.x + NXCD - 1) / NXCD;
    return b;
}

// Wave-wide reservation: lane 0 takes the wave's output range from one of
// the NSH / NXCD shards of the block's XCD sector, picked by the wave's
// position so that the sector's waves spread over them.  No block barrier:
// the waves of a block go on independently.  Every lane of the wave calls it
// with the same total; returns the wave's first output index, `ovf` when the
// range does not fit the shard's region.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t wave_total, const EvDev &E, int type,
                                                 bool &ovf)
{
    const uint32_t x = blockIdx.x % NXCD;
    const uint32_t r = ((blockIdx.x / NXCD) * WAVES + (uint32_t)wave_id()) % (NSH / NXCD);
    const uint32_t shard = x + NXCD * r;
    uint32_t base = 0;
    int o = 0;
    if (lane_id() == 0 && wave_total) {
        base = atomicAdd(&E.gc[gc_shard(type, shard)], wave_total);
        o = ((uint64_t)base + wave_total) > (uint64_t)E.rc[type];
        if (o) atomicOr(&E.gc[GC_OVERFLOW], 1u << type);
    }
    base = __shfl(base, 0, 64);
    ovf = __shfl(o, 0, 64) != 0;
    return shard * E.rc[type] + base;
}

// ---------------------------------------------------------------- zero fill
__device__ __forceinline__ void zero_body(uint4 *p, size_t n16)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_zero(uint4 *p, size_t n16) { zero_body(p, n16); }

hipError_t launch_zero(const EvDev &, void *zero_base, size_t zero_bytes, hipStream_t s)
{
    size_t n16 = zero_bytes / 16;
    int blocks = (int)((n16 + BLOCK - 1) / BLOCK);
    if (blocks > GRID_MAX) blocks = GRID_MAX;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(BLOCK), 0, s, (uint4 *)zero_base, n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------- calibration copy
__global__ __launch_bounds__(BLOCK) void k_copy(uint4 *__restrict__ dst,
                                                const uint4 *__restrict__ src, size_t n16)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) dst[i] = src[i];
}

hipError_t launch_copy(void *dst, const void *src, size_t n_bytes, hipStream_t s)
{
    const size_t n16 = n_bytes / 16;
    // 8 blocks per CU of the 256 CUs, grid-stride
    hipLaunchKernelGGL(k_copy, dim3(2048), dim3(BLOCK), 0, s, (uint4 *)dst, (const uint4 *)src, n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------- hit grouping
__device__ __forceinline__ int event_of(const int32_t *off, int n_ev, int32_t h)
{
    int lo = 0, hi = n_ev - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= h) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int hit_key(const EvDev &E, int n_mod, int n_ev, int32_t h, int &ev)
{
    ev = event_of(E.hit_off, n_ev, h);
    int32_t m = E.module[h];
    uint8_t s = E.sensor[h];
    if (m < 0 || m >= n_mod || s > 1) return -1;
    return 2 * (ev * n_mod + m) + s;
}

// Bin counts per key, and each hit's rank in its bin (the value its atomic
// returned), so that the scatter needs no atomics.  The bins are zero on
// entry: the arena is cleared when it is attached and every scan clears the
// counts it reads.  The same launch clears the chain's counters and the
// scan's tile status, which only later kernels use.
__device__ __forceinline__ void hist_body(const EvDev &E, int n_mod)
{
    const int n_ev = E.desc[D_NEV], n_hits = E.desc[D_NHITS];
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    for (int i = t0; i < GC_COUNT; i += stride) E.gc[i] = 0u;
    const int n_tiles = (E.cap_keys + 1 + SCAN_TILE - 1) / SCAN_TILE;
    for (int i = t0; i < n_tiles; i += stride) E.scan_st[i] = 0ull;
    for (int32_t h = t0; h < n_hits; h += stride) {
        int ev;
        const int key = hit_key(E, n_mod, n_ev, h, ev);
        if (key >= 0) E.hrank[h] = atomicAdd(&E.bcnt[key], 1u);
    }
}

// Exclusive scan of bcnt[0..n) into boff[0..n] in one pass (decoupled
// look-back): a block takes tiles of SCAN_TILE keys in ticket order, publishes
// its tile sum, then walks back over the predecessors' published sums until
// it meets an inclusive prefix.  Status words hold flag and value together,
// so one device-scope atomic load sees both.  A block only ever waits for
// tiles taken before its own, by blocks that are already running.
constexpr unsigned long long ST_AGG = 1ull << 62, ST_INC = 2ull << 62;
constexpr uint32_t SCAN_SPIN_LIMIT = 1u << 20;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &total)
{
    __shared__ uint32_t s_w[WAVES];
    uint32_t incl = wave_incl_scan(v);
    const int w = wave_id();
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

__device__ __forceinline__ void scan_body(const EvDev &E)
{
    __shared__ int s_tile;
    __shared__ uint32_t s_prefix;
    const int n = E.desc[D_NKEYS];
    const int nb = (n + 1 + SCAN_TILE - 1) / SCAN_TILE;   // index n holds the total
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(&E.gc[GC_SCAN], 1u);
        __syncthreads();
        const int tile = s_tile;
        if (tile >= nb) break;
        constexpr int ITEMS = SCAN_TILE / BLOCK;   // consecutive keys per thread
        const int base = tile * SCAN_TILE + threadIdx.x * ITEMS;
        uint32_t v[ITEMS], sum = 0;
        if (base + ITEMS <= n) {
            uint4 *src = reinterpret_cast<uint4 *>(E.bcnt + base);
#pragma unroll
            for (int k = 0; k < ITEMS / 4; ++k) {
                const uint4 q = src[k];
                v[4 * k] = q.x;
                v[4 * k + 1] = q.y;
                v[4 * k + 2] = q.z;
                v[4 * k + 3] = q.w;
                src[k] = make_uint4(0u, 0u, 0u, 0u);   // bins end at zero
            }
        } else {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                v[k] = (base + k < n) ? E.bcnt[base + k] : 0u;
                if (base + k < n) E.bcnt[base + k] = 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) sum += v[k];
        uint32_t tot;
        uint32_t ex = block_excl_scan(sum, tot);
        if (threadIdx.x == 0) {
            unsigned long long *st = E.scan_st;
            uint32_t prefix = 0;
            if (tile == 0) {
                __hip_atomic_store(&st[0], ST_INC | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(&st[tile], ST_AGG | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t it = 0;
                for (int j = tile - 1; j >= 0;) {
                    const unsigned long long w =
                        __hip_atomic_load(&st[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (w & ST_INC) {
                        prefix += (uint32_t)w;
                        break;
                    }
                    if (w & ST_AGG) {
                        prefix += (uint32_t)w;
                        --j;
                        continue;
                    }
                    if (++it > SCAN_SPIN_LIMIT) {   // cannot happen with running predecessors
                        atomicOr(&E.gc[GC_ERROR], 4u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __hip_atomic_store(&st[tile], ST_INC | (uint32_t)(prefix + tot), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            s_prefix = prefix;
        }
        __syncthreads();
        ex += s_prefix;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int idx = base + k;
            if (idx < n) E.boff[idx] = ex;
            if (idx == n) {   // the total, written by the thread covering index n
                E.boff[n] = ex;
                E.gc[GC_N_SORTED] = ex;
            }
            ex += v[k];
        }
        __syncthreads();   // s_tile is rewritten by the next ticket
    }
}

// module frame of module m (half-precision hit storage)
__device__ __forceinline__ ModF mod_frame(const ModDev &M, int m)
{
    ModF f;
    f.cx = M.cx[m]; f.cy = M.cy[m]; f.cz = M.cz[m];
    f.ux = M.ux[m]; f.uy = M.uy[m]; f.uz = M.uz[m];
    f.vx = M.vx[m]; f.vy = M.vy[m]; f.vz = M.vz[m];
    f.wx = M.wx[m]; f.wy = M.wy[m]; f.wz = M.wz[m];
    f.g = M.g[m]; f.rl = M.rl[m];
    f.barrel = M.barrel[m]; f.is2s = M.is2s[m];
    return f;
}

__device__ __forceinline__ void scatter_body(const EvDev &E, const ModDev &M)
{
    const int n_mod = M.n_mod;
    const int n_ev = E.desc[D_NEV], n_hits = E.desc[D_NHITS];
    for (int32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < n_hits;
         h += gridDim.x * blockDim.x) {
        int ev;
        const int key = hit_key(E, n_mod, n_ev, h, ev);
        if (key < 0) {
            atomicOr(&E.gc[GC_ERROR], 1u);
            continue;
        }
        const uint32_t pos = E.boff[key] + E.hrank[h];
        if (pos >= (uint32_t)E.cap_hits) {   // inconsistent grouping: never written
            atomicOr(&E.gc[GC_ERROR], 4u);
            continue;
        }
        // one 16-byte store per hit (scattered 4-byte stores cost a line each),
        // or one 8-byte record in half-precision storage
        if (E.half16)
            E.hsort_h[pos] = half_hit(mod_frame(M, E.module[h]), E.x[h], E.y[h], E.z[h], h - E.hit_off[ev]);
        else
            E.hsort[pos] = make_float4(E.x[h], E.y[h], E.z[h], __int_as_float(h - E.hit_off[ev]));
    }
}

__global__ void k_hist(EvDev E, int n_mod) { hist_body(E, n_mod); }

__global__ __launch_bounds__(BLOCK) void k_scan(EvDev E) { scan_body(E); }
__global__ void k_scatter(EvDev E, ModDev M) { scatter_body(E, M); }

// Batches: each event's 2 x n_mod bins are split in SORT_EV_PARTS ranges of
// consecutive keys; one block per (event, range) keeps its bins in LDS and
// takes the event's hits whose key falls in its range, so the histogram and
// the scatter use LDS atomics instead of device-scope ones.  Same results as
// the kernels above (bin counts, then the same look-back scan, then each hit
// to a slot of its bin), and the bins end at zero as they do there.
constexpr int SORT_EV_BLOCK = 1024;
constexpr int SORT_EV_ILP = 4;
constexpr int SORT_EV_PARTS = 4;

__device__ __forceinline__ int sort_ev_span(int nk) { return (nk + SORT_EV_PARTS - 1) / SORT_EV_PARTS; }

__global__ __launch_bounds__(SORT_EV_BLOCK) void k_hist_ev(EvDev E, int n_mod)
{
    extern __shared__ uint32_t s_bin[];     // [sort_ev_span(2 n_mod)]
    const int n_ev = E.desc[D_NEV], nk = 2 * n_mod, kp = sort_ev_span(nk);
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    for (int i = t0; i < GC_COUNT; i += stride) E.gc[i] = 0u;
    const int n_tiles = (E.cap_keys + 1 + SCAN_TILE - 1) / SCAN_TILE;
    for (int i = t0; i < n_tiles; i += stride) E.scan_st[i] = 0ull;
    for (int item = blockIdx.x; item < n_ev * SORT_EV_PARTS; item += gridDim.x) {
        const int ev = item / SORT_EV_PARTS, k0 = (item - ev * SORT_EV_PARTS) * kp;
        const int k1 = k0 + kp < nk ? k0 + kp : nk;
        for (int k = threadIdx.x; k < k1 - k0; k += blockDim.x) s_bin[k] = 0u;
        __syncthreads();
        const int h1 = E.hit_off[ev + 1];
        // SORT_EV_ILP hits per thread and step: their loads are issued together
        for (int hb = E.hit_off[ev] + threadIdx.x; hb < h1; hb += SORT_EV_ILP * blockDim.x) {
            int32_t m[SORT_EV_ILP];
            uint8_t sn[SORT_EV_ILP];
#pragma unroll
            for (int u = 0; u < SORT_EV_ILP; ++u) {
                const int h = hb + u * (int)blockDim.x;
                m[u] = h < h1 ? E.module[h] : -1;
                sn[u] = h < h1 ? E.sensor[h] : 0;
            }
#pragma unroll
            for (int u = 0; u < SORT_EV_ILP; ++u) {
                const int key = 2 * m[u] + sn[u];
                if (m[u] >= 0 && m[u] < n_mod && sn[u] <= 1 && key >= k0 && key < k1)
                    atomicAdd(&s_bin[key - k0], 1u);
            }
        }
        __syncthreads();
        uint32_t *dst = E.bcnt + (size_t)nk * ev;
        for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) dst[k] = s_bin[k - k0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(SORT_EV_BLOCK) void k_scatter_ev(EvDev E, ModDev M)
{
    const int n_mod = M.n_mod;
    extern __shared__ uint32_t s_cur[];     // next free slot of each bin of the range
    const int n_ev = E.desc[D_NEV], nk = 2 * n_mod, kp = sort_ev_span(nk);
    for (int item = blockIdx.x; item < n_ev * SORT_EV_PARTS; item += gridDim.x) {
        const int ev = item / SORT_EV_PARTS, part = item - ev * SORT_EV_PARTS, k0 = part * kp;
        const int k1 = k0 + kp < nk ? k0 + kp : nk;
        const uint32_t *off = E.boff + (size_t)nk * ev;
        for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) s_cur[k - k0] = off[k];
        __syncthreads();
        const int h0 = E.hit_off[ev], h1 = E.hit_off[ev + 1];
        for (int hb = h0 + threadIdx.x; hb < h1; hb += SORT_EV_ILP * blockDim.x) {
            int key[SORT_EV_ILP];
#pragma unroll
            for (int u = 0; u < SORT_EV_ILP; ++u) {
                const int h = hb + u * (int)blockDim.x;
                key[u] = -1;
                if (h < h1) {
                    const int32_t m = E.module[h];
                    const uint8_t sn = E.sensor[h];
                    if (m < 0 || m >= n_mod || sn > 1) {
                        if (part == 0) atomicOr(&E.gc[GC_ERROR], 1u);
                    } else {
                        key[u] = 2 * m + sn;
                    }
                }
            }
            float4 v[SORT_EV_ILP];
#pragma unroll
            for (int u = 0; u < SORT_EV_ILP; ++u) {
                const int h = hb + u * (int)blockDim.x;
                if (key[u] >= k0 && key[u] < k1)
                    v[u] = make_float4(E.x[h], E.y[h], E.z[h], __int_as_float(h - h0));
            }
#pragma unroll
            for (int u = 0; u < SORT_EV_ILP; ++u) {
                if (key[u] >= k0 && key[u] < k1) {
                    const uint32_t pos = atomicAdd(&s_cur[key[u] - k0], 1u);
                    if (E.half16)
                        E.hsort_h[pos] = half_hit(mod_frame(M, key[u] >> 1), v[u].x, v[u].y, v[u].z,
                                                  __float_as_int(v[u].w));
                    else
                        E.hsort[pos] = v[u];
                }
            }
        }
        // the bins end at zero, as the device-wide scatter leaves them
        uint32_t *bc = E.bcnt + (size_t)nk * ev;
        for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) bc[k] = 0u;
        __syncthreads();
    }
}

size_t sort_ev_lds_bytes(int n_mod)
{
    return (size_t)((2 * n_mod + SORT_EV_PARTS - 1) / SORT_EV_PARTS) * sizeof(uint32_t);
}

hipError_t sort_ev_prepare(int n_mod)
{
    const int bytes = (int)sort_ev_lds_bytes(n_mod);
    hipError_t e = hipFuncSetAttribute((const void *)k_hist_ev,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_scatter_ev,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// grids depend on the arena capacities only, never on the batch
hipError_t launch_sort(const EvDev &E, const ModDev &M, int grid, bool per_event, hipStream_t s)
{
    const int nb = (E.cap_keys + 1 + SCAN_TILE - 1) / SCAN_TILE;
    if (per_event) {
        const int items = E.cap_ev * SORT_EV_PARTS;
        const int eg = items < GRID_MAX ? items : GRID_MAX;
        const size_t lds = sort_ev_lds_bytes(M.n_mod);
        hipLaunchKernelGGL(k_hist_ev, dim3(eg), dim3(SORT_EV_BLOCK), lds, s, E, M.n_mod);
        hipLaunchKernelGGL(k_scan, dim3(nb < 1024 ? nb : 1024), dim3(BLOCK), 0, s, E);
        hipLaunchKernelGGL(k_scatter_ev, dim3(eg), dim3(SORT_EV_BLOCK), lds, s, E, M);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_hist, dim3(grid), dim3(BLOCK), 0, s, E, M.n_mod);
    hipLaunchKernelGGL(k_scan, dim3(nb < 1024 ? nb : 1024), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(BLOCK), 0, s, E, M);
    return hipGetLastError();
}

// ---------------------------------------------------------------- LDS layouts
// segment stage: per wave, the queue of window survivors (see enum_seg)
constexpr int SEGQ = 128;             // ring entries: a full wave plus what is pending
constexpr int MAXP = 64 / 8;          // groups per wave at the narrowest width
struct SegQ {
    float4 ip[MAXP], id[MAXP];        // inner MD of each group (SegIn)
    float4 w0[MAXP], w1[MAXP];        // its window terms (x, y, r, a), (ca, 1/r, |sv|/r, -)
    int2 eb[MAXP];                    // its module's first map edge, its event's first slot
    int32_t ib[MAXP], idx[MAXP], off[MAXP];
    int32_t o[SEGQ], o2[SEGQ];        // window survivors; angle survivors
    int32_t mark[64];                 // chunk_src
    uint8_t g[SEGQ], g2[SEGQ];
    uint8_t nf[MAXP];                 // groups sharing a leading group's candidates
};

// mini-doublet stage: accepted pairs and their window outputs staged until
// the output offset is known
struct ModL {
    float4 c, u, v;                   // (cx, cy, cz, g), (ux, uy, uz, rl), (vx, vy, vz, flags)
    float4 w;                         // (wx, wy, wz, -): sensor normal
};
struct SmMD {
    uint32_t lo[WAVES][STAGE], up[WAVES][STAGE];
    float bend[WAVES][STAGE], sv[WAVES][STAGE];
    ModL mod[WAVES][MAXP];            // module frame of each group's slot
    int4 sl[WAVES][MAXP];             // slot, first lower hit, first upper hit, upper hits
    int4 nb[WAVES][MAXP];             // the slot's map row and its event's first slot
    uint32_t cnt[WAVES][MAXP];
    uint8_t g[WAVES][STAGE];
};
struct SmSeg {
    int32_t o[WAVES][STAGE];
    SegQ q[WAVES];
};
// triplet stage: per wave, the inner MDs of the round (one per lane) and the
// accepted triplets staged until their output offset is known
constexpr int T3_PMAX = 32;           // most inner MDs a wave takes per round
struct SmT3 {
    int32_t b[WAVES][STAGE], c[WAVES][STAGE];
    float k[WAVES][STAGE];
    float4 ap[WAVES][T3_PMAX];        // inner MD anchor (x, y, z, r)
    float asv[WAVES][T3_PMAX];        // its sv
    int32_t abar[WAVES][T3_PMAX], aidx[WAVES][T3_PMAX];
    uint32_t cnt[WAVES][T3_PMAX];
    int32_t mark[WAVES][64];          // chunk_src
    uint8_t g[WAVES][STAGE];
};
// quintuplet stage: the same per-wave table of inner MDs and staging
constexpr int T5_PMAX = 32;
struct SmT5 {
    int32_t b[WAVES][STAGE], c[WAVES][STAGE], d[WAVES][STAGE], e[WAVES][STAGE];
    float s[WAVES][STAGE];
    float4 ap[WAVES][T5_PMAX];
    float asv[WAVES][T5_PMAX];
    int32_t abar[WAVES][T5_PMAX], aidx[WAVES][T5_PMAX];
    uint32_t cnt[WAVES][T5_PMAX];     // accepted quintuplets per inner MD
    int32_t mark[WAVES][64];          // chunk_src
    uint8_t g[WAVES][STAGE];
};
struct SmChain {
    union {
        SmMD md;
        SmSeg seg;
        SmT3 t3;
        SmT5 t5;
    } u;
    uint32_t pre[NSH + 1];
};

// ---------------------------------------------------------------- mini-doublets
__device__ __forceinline__ void write_md(const EvDev &E, const Consts &K, uint32_t i, int slot,
                                         uint32_t hl, uint32_t hu, const MdOut &o,
                                         const ModF &mod, const int4 &nbr)
{
    const float4 L = stored_hit(E, mod, hl, 0), U = stored_hit(E, mod, hu, 1);
    const float xL = L.x, yL = L.y;
    E.md_hlo[i] = (int32_t)hl;
    E.md_hup[i] = (int32_t)hu;
    E.md_slot[i] = slot;
    E.md_nbr[i] = nbr;
    const float dx = U.x - xL, dy = U.y - yL;
    E.md_p0[i] = make_float4(xL, yL, L.z, o.r);
    // the segment window's per-MD terms, rounded exactly as it would round them
    E.md_p1[i] = make_float4(o.a, o.ca, 1.0f / o.r, fabsf(o.sv) / o.r);
    const float dn = sqrtf((dx * dx) + (dy * dy));
    E.md_p2[i] = make_float4(dx, dy, dn, o.sv);
    E.md_atol[i] = seg_angle_bound(K, dn);
    E.md_bend[i] = o.bend;
    E.md_bar[i] = (uint8_t)(mod.barrel | (mod.is2s << 1));
}

__device__ __forceinline__ ModF mod_from(const ModL &r)
{
    ModF f;
    f.cx = r.c.x; f.cy = r.c.y; f.cz = r.c.z; f.g = r.c.w;
    f.ux = r.u.x; f.uy = r.u.y; f.uz = r.u.z; f.rl = r.u.w;
    f.vx = r.v.x; f.vy = r.v.y; f.vz = r.v.z;
    const int fl = __float_as_int(r.v.w);
    f.barrel = fl & 1;
    f.is2s = fl >> 1;
    f.wx = r.w.x; f.wy = r.w.y; f.wz = r.w.z;
    return f;
}

// Every lower x upper hit pair of the wave's P module slots (one per group,
// its frame and hit ranges in the LDS table), walked as one list 64 pairs at
// a time, so a slot with many hits is shared by all lanes of the wave.  The
// list is in slot order, so each slot's accepted pairs are consecutive in
// the wave's output, in lower-major pair order.
// sink(ok, g, hl, hu, o, pos): g = group of the slot, pos = rank among the
// wave's accepted pairs, o the window's outputs for the pair.
template <int G, class F>
__device__ __forceinline__ uint32_t enum_md(const EvDev &E, const Consts &K, const SmMD &sm, int w,
                                            uint32_t np, F &&sink)
{
    constexpr int P = Grp<G>::P;
    const uint32_t l = (uint32_t)lane_id();
    const unsigned long long below = lanes_below();
    uint32_t pre[P + 1];
    pre[0] = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
        pre[p + 1] = pre[p] + (uint32_t)__builtin_amdgcn_readlane((int)np, p * G);
    const uint32_t tot = pre[P];
    uint32_t acc = 0;
    for (uint32_t jc = 0; jc < tot; jc += 64) {
        const uint32_t j = jc + l;
        int g = 0;
        uint32_t gpre = 0;
#pragma unroll
        for (int p = 1; p < P; ++p)
            if (j >= pre[p]) {
                g = p;
                gpre = pre[p];
            }
        bool ok = false;
        uint32_t hl = 0, hu = 0;
        MdOut o = {};
        if (j < tot) {
            const int4 sl = sm.sl[w][g];
            const uint32_t p = j - gpre, nup = (uint32_t)sl.w;
            const uint32_t il = p / nup, iu = p - il * nup;
            hl = (uint32_t)sl.y + il;
            hu = (uint32_t)sl.z + iu;
            const ModF mf = mod_from(sm.mod[w][g]);
            const float4 L = stored_hit(E, mf, hl, 0), U = stored_hit(E, mf, hu, 1);
            ok = md_accept(K, mf, L.x, L.y, L.z, U.x, U.y, U.z, o);
        }
        const unsigned long long m = __ballot(ok);
        sink(ok, g, hl, hu, o, acc + (uint32_t)__popcll(m & below));
        acc += (uint32_t)__popcll(m);
    }
    return acc;
}

// one group of G lanes per module slot sets it up; the pairs are walked by
// the whole wave
template <int G>
__device__ __forceinline__ void md_body(const EvDev &E, const ModDev &M, const Consts &K, SmMD &sm)
{
    constexpr int P = Grp<G>::P;
    const Grp<G> gp;
    const int w = wave_id();
    const uint32_t l = (uint32_t)lane_id();
    const XBlock xb = xcd_block();
    const int n_x = M.sec_off[xb.x + 1] - M.sec_off[xb.x];   // modules of this sector
    const int items = E.desc[D_NEV] * n_x;
    // one pass over the sector: group g of wave slot u takes the u-th module
    // of the sector's g-th run (spreads the dense modules over the waves, as
    // in the segment stage), else consecutive modules
    const int nslot = (items + P - 1) / P;
    const bool spread = nslot <= (int)xb.count * WAVES;
    for (int base = (int)xb.rank * WAVES; base < nslot; base += (int)xb.count * WAVES) {
        const int u = base + w;
        const int k = spread ? gp.g * nslot + u : u * P + gp.g;
        const bool act = u < nslot && k < items;
        int slot = 0;
        uint32_t lo0 = 0, up0 = 0, nup = 0, np = 0;
        if (act) {
            const int ev = k / n_x;
            const int m = M.xorder[M.sec_off[xb.x] + (k - ev * n_x)];
            slot = ev * M.n_mod + m;
            lo0 = E.boff[2 * slot];
            up0 = E.boff[2 * slot + 1];
            nup = E.boff[2 * slot + 2] - up0;
            np = (up0 - lo0) * nup;
            // per-hit state of duplicate removal for this slot's hits (contiguous)
            for (uint32_t h = lo0 + gp.lane; h < up0 + nup; h += G) {
                E.hmin[h] = 0xffffffffu;
                E.htie[h] = 0;
                E.thead[h] = 0;
            }
            if (gp.lane == 0) {
                sm.sl[w][gp.g] = make_int4(slot, (int)lo0, (int)up0, (int)nup);
                const int e0 = M.map_ptr[m];
                sm.nb[w][gp.g] = make_int4(e0, M.map_ptr[m + 1] - e0, ev * M.n_mod, 0);
                if (np) {
                    ModL r;
                    r.c = make_float4(M.cx[m], M.cy[m], M.cz[m], M.g[m]);
                    r.u = make_float4(M.ux[m], M.uy[m], M.uz[m], M.rl[m]);
                    r.v = make_float4(M.vx[m], M.vy[m], M.vz[m],
                                      __int_as_float(M.barrel[m] | (M.is2s[m] << 1)));
                    r.w = make_float4(M.wx[m], M.wy[m], M.wz[m], 0.0f);
                    sm.mod[w][gp.g] = r;
                }
            }
        }
        if (l < (uint32_t)MAXP) sm.cnt[w][l] = 0u;
        wave_lds_sync();
        const uint32_t tot = enum_md<G>(E, K, sm, w, np,
                                        [&](bool ok, int g, uint32_t hl, uint32_t hu, const MdOut &o,
                                            uint32_t pos) {
            if (ok) {
                atomicAdd(&sm.cnt[w][g], 1u);
                if (pos < STAGE) {
                    sm.lo[w][pos] = hl;
                    sm.up[w][pos] = hu;
                    sm.bend[w][pos] = o.bend;
                    sm.sv[w][pos] = o.sv;
                    sm.g[w][pos] = (uint8_t)g;
                }
            }
        });
        wave_lds_sync();
        // each slot's MDs follow those of the groups before it
        const uint32_t cnt = act ? sm.cnt[w][gp.g] : 0u;
        uint32_t wtot;
        const uint32_t gex = gp.wave_prefix(cnt, wtot);
        bool ovf;
        const uint32_t off = wave_reserve(tot, E, OT_MD, ovf);
        if (act && gp.lane == 0) {
            E.md_start[slot] = (int32_t)(off + gex);
            E.md_cnt[slot] = ovf ? 0 : (int32_t)cnt;
        }
        if (ovf) continue;
        for (uint32_t q = l; q < tot && q < (uint32_t)STAGE; q += 64) {
            const int g = sm.g[w][q];
            const uint32_t hl = sm.lo[w][q];
            const float4 L = stored_hit(E, mod_from(sm.mod[w][g]), hl, 0);
            MdOut o;
            md_anchor(K, L.x, L.y, o);
            o.bend = sm.bend[w][q];
            o.sv = sm.sv[w][q];
            write_md(E, K, off + q, sm.sl[w][g].x, hl, sm.up[w][q], o, mod_from(sm.mod[w][g]), sm.nb[w][g]);
        }
        if (tot > (uint32_t)STAGE) {
            // beyond the staging: enumerate again and write directly
            enum_md<G>(E, K, sm, w, np,
                       [&](bool ok, int g, uint32_t hl, uint32_t hu, const MdOut &o, uint32_t pos) {
                if (ok && pos >= STAGE)
                    write_md(E, K, off + pos, sm.sl[w][g].x, hl, hu, o, mod_from(sm.mod[w][g]), sm.nb[w][g]);
            });
        }
        wave_lds_sync();
    }
}

template <int G>
__global__ __launch_bounds__(BLOCK, 6) void k_md(EvDev E, ModDev M, Consts K)
{
    __shared__ SmMD sm;
    md_body<G>(E, M, K, sm);
}

// the group widths a stage kernel is built for
// object-stage grids: at least one block per sector, whole rounds of sectors
static int xcd_grid(int grid) { return grid < NXCD ? NXCD : (grid + NXCD - 1) / NXCD * NXCD; }

#define LST_BY_LANES(lanes, KERNEL, ...)                                              \
    switch (lanes) {                                                                  \
    case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                        \
    case 16: hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__); break;                      \
    case 32: hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__); break;                      \
    default: hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__); break;                      \
    }

hipError_t launch_md(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                     hipStream_t s)
{
    LST_BY_LANES(lanes, k_md, dim3(xcd_grid(grid)), dim3(BLOCK), 0, s, E, M, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- segments

// Outer candidates of inner MD i: the MDs of every map edge of its module,
// in edge order; the candidates of the wave's inner MDs are walked as one
// list.  The pairs inside the azimuth window (about a third of them) go to a
// ring of the wave in LDS; 64 queued pairs at a time take the angle cut,
// whose survivors queue again for the pointing cut, so each costly part of
// the test runs on full waves of the pairs that reached it.  The rings keep
// the enumeration order, so accepted pairs get, per inner MD, consecutive
// positions in that order.  sink(g, ok, o, pos): g is the group of the
// pair's inner MD.
template <int G, bool SHARE, class F>
__device__ __forceinline__ uint32_t enum_seg(const EvDev &E, const ModDev &M, const Consts &K,
                                             int32_t i, bool act, SegQ &q, F &&sink)
{
    constexpr int P = Grp<G>::P;
    const Grp<G> gp;
    const Grp<64> gw;
    const uint32_t l = (uint32_t)lane_id();
    int4 nb = make_int4(-1, 0, -1, 0);
    if (act) {
        nb = E.md_nbr[i];
        const int32_t e0 = nb.x;
        if (gp.lane == 0) {
            const float4 p0 = E.md_p0[i], p1 = E.md_p1[i], p2 = E.md_p2[i];
            q.ip[gp.g] = p0;
            q.id[gp.g] = make_float4(p2.x, p2.y, p2.z, E.md_atol[i]);
            q.ib[gp.g] = E.md_bar[i] & 1;
            q.w0[gp.g] = make_float4(p0.x, p0.y, p0.w, p1.x);
            q.w1[gp.g] = make_float4(p1.y, p1.z, p1.w, 0.0f);
            q.eb[gp.g] = make_int2(e0, nb.z);
        }
    }
    // Groups whose inner MDs lie in one module (next to each other in the
    // regions) have the same candidates: the first of a run of such groups
    // enumerates them and each candidate is tested against every MD of the
    // run.  A module is keyed by its map row and its event.
    // (SHARE: the wave's inner MDs are consecutive in their region, else
    // they come from distant parts of it and every group leads)
    uint32_t ne_of[P];
    int nmax = 1;
    if constexpr (SHARE) {
        int lead[P], nfol[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int32_t kx = __builtin_amdgcn_readlane(nb.x, p * G);
            const int32_t ky = __builtin_amdgcn_readlane(nb.y, p * G);
            const int32_t kz = __builtin_amdgcn_readlane(nb.z, p * G);
            lead[p] = p;
            if (p > 0 && kx >= 0 && kx == __builtin_amdgcn_readlane(nb.x, (p - 1) * G) &&
                ky == __builtin_amdgcn_readlane(nb.y, (p - 1) * G) &&
                kz == __builtin_amdgcn_readlane(nb.z, (p - 1) * G))
                lead[p] = lead[p - 1];
            ne_of[p] = lead[p] == p ? (uint32_t)ky : 0u;
            nfol[p] = 0;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int r = 0; r < P; ++r)
                if (lead[r] == p) ++nfol[p];
            nmax = nfol[p] > nmax ? nfol[p] : nmax;
            if (l == 0) q.nf[p] = (uint8_t)nfol[p];
        }
    } else {
#pragma unroll
        for (int p = 0; p < P; ++p) ne_of[p] = (uint32_t)__builtin_amdgcn_readlane(nb.y, p * G);
    }
    // the wave's (leading inner MD, map edge) pairs as one list in group
    // order: pre[g] = edges of the groups before g
    uint32_t pre[P + 1];
    pre[0] = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) pre[p + 1] = pre[p] + ne_of[p];
    const uint32_t n_edges = pre[P];
    uint32_t cnt[P];
#pragma unroll
    for (int p = 0; p < P; ++p) cnt[p] = 0;
    uint32_t head = 0, tail = 0;                  // ring positions (wave-uniform)
    const unsigned long long below = lanes_below();
    wave_lds_sync();
    uint32_t head2 = 0, tail2 = 0;
    // the pointing cut on the n (<= 64) oldest angle survivors: final decision
    auto drain2 = [&](uint32_t n) {
        wave_lds_sync();
        bool ok = false;
        int32_t o = 0;
        int g = 0;
        if (l < n) {
            const uint32_t s = (head2 + l) & (SEGQ - 1);
            o = q.o2[s];
            g = q.g2[s];
            SegIn I;
            I.p = q.ip[g];
            I.d = q.id[g];
            I.barrel = q.ib[g];
            ok = seg_point(K, I, E, o);
        }
        head2 += n;
        uint32_t pos = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const unsigned long long mk = __ballot(ok && g == p);
            if (g == p) pos = cnt[p] + (uint32_t)__popcll(mk & below);
            cnt[p] += (uint32_t)__popcll(mk);
        }
        sink(g, ok, o, pos);
        wave_lds_sync();                          // slots are rewritten by later pairs
    };
    // the angle cut on the n (<= 64) oldest window survivors; its survivors
    // queue for the pointing cut in the same order
    auto drain = [&](uint32_t n) {
        wave_lds_sync();
        bool ok = false;
        int32_t o = 0;
        int g = 0;
        if (l < n) {
            const uint32_t s = (head + l) & (SEGQ - 1);
            o = q.o[s];
            g = q.g[s];
            SegIn I;
            I.p = q.ip[g];
            I.d = q.id[g];
            I.barrel = q.ib[g];
            ok = seg_angle(I, E, o);
        }
        head += n;
        const unsigned long long mk = __ballot(ok);
        if (ok) {
            const uint32_t s = (tail2 + (uint32_t)__popcll(mk & below)) & (SEGQ - 1);
            q.o2[s] = o;
            q.g2[s] = (uint8_t)g;
        }
        tail2 += (uint32_t)__popcll(mk);
        if (tail2 - head2 >= 64) drain2(64);
        wave_lds_sync();
    };
    // 64 (MD, edge) pairs at a time: their candidates (the MDs of the edge's
    // module) as one list the 64 lanes walk 64 at a time
    for (uint32_t fc = 0; fc < n_edges; fc += 64) {
        const uint32_t f = fc + l;
        int ge = 0;
        uint32_t gpre = 0;
#pragma unroll
        for (int p = 1; p < P; ++p)
            if (f >= pre[p]) {
                ge = p;
                gpre = pre[p];
            }
        uint32_t bc = 0;
        int32_t bs = 0;
        if (f < n_edges) {
            const int2 eb = q.eb[ge];
            const int b = eb.y + M.map_col[eb.x + (int32_t)(f - gpre)];
            bs = E.md_start[b];
            bc = (uint32_t)E.md_cnt[b];
        }
        const uint32_t incl = wave_incl_scan(bc);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        // candidate jc + l of the list: its outer MD o and the group g of its
        // inner MD; the outer anchors are loaded one chunk of 64 ahead, so
        // their latency overlaps the window test and queueing of the chunk
        // before
        auto locate = [&](uint32_t jc, int32_t &o, int &g) {
            const int src = chunk_src(incl, bc, jc, q.mark);
            const uint32_t ex = gw.bcast(incl, src) - gw.bcast(bc, src);
            o = gw.bcast(bs, src) + (int32_t)(jc + l - ex);
            g = gw.bcast(ge, src);
            return jc + l < tot;
        };
        int32_t o = 0;
        int g = 0;
        bool live = false;
        float4 a0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), a1 = a0;
        if (tot > 0) {
            live = locate(0, o, g);
            if (live) {
                a0 = E.md_p0[o];
                a1 = E.md_p1[o];
            }
        }
        for (uint32_t jc = 0; jc < tot; jc += 64) {
            int32_t on = 0;
            int gn = 0;
            bool ln = false;
            float4 b0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), b1 = b0;
            if (jc + 64 < tot) {
                ln = locate(jc + 64, on, gn);
                if (ln) {
                    b0 = E.md_p0[on];
                    b1 = E.md_p1[on];
                }
            }
            // the candidate against each inner MD of its run of groups
            const int nf = live ? (SHARE ? (int)q.nf[g] : 1) : 0;
            for (int k = 0; k < (SHARE ? nmax : 1); ++k) {
                bool win = false;
                if (k < nf) {
                    const float4 w0 = q.w0[g + k], w1 = q.w1[g + k];
                    win = seg_window(K, w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, a0, a1);
                }
                const unsigned long long mk = __ballot(win);
                if (win) {
                    const uint32_t s = (tail + (uint32_t)__popcll(mk & below)) & (SEGQ - 1);
                    q.o[s] = o;
                    q.g[s] = (uint8_t)(g + k);
                }
                tail += (uint32_t)__popcll(mk);
                if (tail - head >= 64) drain(64);
            }
            o = on;
            g = gn;
            live = ln;
            a0 = b0;
            a1 = b1;
        }
    }
    if (tail != head) drain(tail - head);
    if (tail2 != head2) drain2(tail2 - head2);
    uint32_t c = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (gp.g == p) c = cnt[p];
    return c;
}

// SHARE: runs of inner MDs of one module may share their candidate
// enumeration (when the order is consecutive); else every group enumerates
// its own (the single-event kernel, whose one-pass order spreads the MDs)
template <int G, bool SHARE>
__device__ __forceinline__ void seg_body(const EvDev &E, const ModDev &M, const Consts &K, SmSeg &sm)
{
    if (upstream_overflow(E)) return;
    constexpr int P = Grp<G>::P, CAP = STAGE / P;
    const Grp<G> gp;
    const int w = wave_id();
    SegQ &q = sm.q[w];
    const XBlock xb = xcd_block();
    const XRegions R = load_regions_x(E, OT_MD, xb.x);
    // MDs of one module (same map edges, same candidate count) sit next to
    // each other in the regions, so P consecutive MDs in one wave add up a
    // dense module's load P times.  When the grid covers the sector in one
    // pass, the longest wave sets the kernel's duration: the sector's MDs are
    // then split into P equal runs and group g of wave slot u takes the u-th
    // MD of run g, which evens out the waves' lengths.  Over several passes
    // the lengths average out and consecutive MDs keep their shared
    // candidates in the caches.
    const uint32_t nslot = (R.total + P - 1) / P;
    const bool spread = nslot <= xb.count * WAVES;
    for (uint32_t base = xb.rank * WAVES; base < nslot; base += xb.count * WAVES) {
        const uint32_t u = base + (uint32_t)w;
        const uint32_t v = spread ? (uint32_t)gp.g * nslot + u : u * P + (uint32_t)gp.g;
        const bool act = u < nslot && v < R.total;
        const int32_t i = region_index_x(R, act ? v : 0);
        auto stage = [&](int g, bool ok, int32_t o, uint32_t pos) {
            if (ok && pos < CAP) sm.o[w][g * CAP + pos] = o;
        };
        // consecutive inner MDs (several passes): runs of one module share
        // their candidate enumeration
        uint32_t cnt;
        if constexpr (SHARE)
            cnt = spread ? enum_seg<G, false>(E, M, K, i, act, q, stage)
                         : enum_seg<G, true>(E, M, K, i, act, q, stage);
        else
            cnt = enum_seg<G, false>(E, M, K, i, act, q, stage);
        uint32_t wtot;
        const uint32_t gex = gp.wave_prefix(cnt, wtot);
        bool ovf;
        const uint32_t off = wave_reserve(wtot, E, OT_SEG, ovf) + gex;
        if (act && gp.lane == 0) {
            E.seg_start[i] = (int32_t)off;
            E.seg_cnt[i] = ovf ? 0 : (int32_t)cnt;
        }
        if (ovf) continue;
        if (act && cnt <= CAP) {
            for (uint32_t k = gp.lane; k < cnt; k += G) {
                E.seg_in[off + k] = i;
                E.seg_out[off + k] = sm.o[w][gp.g * CAP + k];
            }
        }
        if (wave_max(cnt) > CAP) {
            // groups beyond their staging share enumerate again and write directly
            if (gp.lane == 0) {
                q.idx[gp.g] = i;
                q.off[gp.g] = (int32_t)off;
            }
            auto direct = [&](int g, bool ok, int32_t o, uint32_t pos) {
                if (ok) {
                    E.seg_in[q.off[g] + pos] = q.idx[g];
                    E.seg_out[q.off[g] + pos] = o;
                }
            };
            if constexpr (SHARE) {
                if (spread)
                    enum_seg<G, false>(E, M, K, i, act && cnt > CAP, q, direct);
                else
                    enum_seg<G, true>(E, M, K, i, act && cnt > CAP, q, direct);
            } else {
                enum_seg<G, false>(E, M, K, i, act && cnt > CAP, q, direct);
            }
        }
    }
}

template <int G>
__global__ __launch_bounds__(BLOCK, 6) void k_seg(EvDev E, ModDev M, Consts K)
{
    __shared__ SmSeg sm;
    seg_body<G, false>(E, M, K, sm);
}

template <int G>
__global__ __launch_bounds__(BLOCK, 6) void k_seg_share(EvDev E, ModDev M, Consts K)
{
    __shared__ SmSeg sm;
    seg_body<G, true>(E, M, K, sm);
}

hipError_t launch_seg(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                      bool share, hipStream_t s)
{
    if (share) {
        LST_BY_LANES(lanes, k_seg_share, dim3(xcd_grid(grid)), dim3(BLOCK), 0, s, E, M, K);
    } else {
        LST_BY_LANES(lanes, k_seg, dim3(xcd_grid(grid)), dim3(BLOCK), 0, s, E, M, K);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- triplets
// Candidates of inner MD a: every segment (a->b) followed by every segment
// (b->c).  A wave takes P inner MDs per round, lane l < P holding MD l; their
// first segments, then the candidates, are walked as one list 64 at a time,
// so no lane waits for the MD with most candidates.  The list is in MD order,
// so each MD's accepted triplets are consecutive in the wave's output, in
// enumeration order.  sink(ok, g, b, c, k, pos): g = lane of the inner MD,
// pos = rank among the wave's accepted triplets.
template <class F>
__device__ __forceinline__ uint32_t enum_t3(const EvDev &E, const Consts &K, SmT3 &sm,
                                            int w, int32_t ns1, int32_t s10, uint32_t incl1,
                                            F &&sink)
{
    const Grp<64> gw;
    const uint32_t l = (uint32_t)lane_id();
    const unsigned long long below = lanes_below();
    const uint32_t n1 = (uint32_t)__builtin_amdgcn_readlane((int)incl1, 63);
    uint32_t acc = 0;
    for (uint32_t fc = 0; fc < n1; fc += 64) {
        const uint32_t f = fc + l;
        const int g = chunk_src(incl1, (uint32_t)ns1, fc, sm.mark[w]);
        const uint32_t ex1 = gw.bcast(incl1, g) - gw.bcast((uint32_t)ns1, g);
        const int32_t s10g = gw.bcast(s10, g);
        int32_t b = 0, bs = 0;
        uint32_t nb = 0;
        if (f < n1) {
            b = E.seg_out[s10g + (int32_t)(f - ex1)];
            bs = E.seg_start[b];
            nb = (uint32_t)E.seg_cnt[b];
        }
        const uint32_t incl2 = wave_incl_scan(nb);
        const uint32_t n2 = (uint32_t)__builtin_amdgcn_readlane((int)incl2, 63);
        for (uint32_t jc = 0; jc < n2; jc += 64) {
            const uint32_t j = jc + l;
            const int src = chunk_src(incl2, nb, jc, sm.mark[w]);
            const uint32_t ex2 = gw.bcast(incl2, src) - gw.bcast(nb, src);
            const int32_t bb = gw.bcast(b, src), bbs = gw.bcast(bs, src);
            const int gg = gw.bcast(g, src);
            bool ok = false;
            int32_t c = 0;
            float kk = 0.0f;
            if (j < n2) {
                c = E.seg_out[bbs + (int32_t)(j - ex2)];
                MdV A = {};
                const float4 ap = sm.ap[w][gg];
                A.x = ap.x; A.y = ap.y; A.z = ap.z; A.r = ap.w;
                A.sv = sm.asv[w][gg];
                A.barrel = sm.abar[w][gg];
                ok = t3_accept(K, A, load_md(E, bb), load_md(E, c), kk);
            }
            const unsigned long long m = __ballot(ok);
            sink(ok, gg, bb, c, kk, acc + (uint32_t)__popcll(m & below));
            acc += (uint32_t)__popcll(m);
        }
    }
    return acc;
}

// G selects P = 256 / G inner MDs per wave and round (G = 8: 32 MDs)
template <int G>
__device__ __forceinline__ void t3_body(const EvDev &E, const Consts &K, SmT3 &sm)
{
    if (upstream_overflow(E)) return;
    constexpr int P = 256 / G;
    static_assert(P <= T3_PMAX, "inner MDs per wave");
    const int w = wave_id();
    const uint32_t l = (uint32_t)lane_id();
    const XBlock xb = xcd_block();
    const XRegions R = load_regions_x(E, OT_MD, xb.x);
    // one pass over the sector: lane l of wave slot u takes the u-th MD of the
    // sector's l-th run (as in the segment stage), else consecutive MDs
    const uint32_t nslot = (R.total + P - 1) / P;
    const bool spread = nslot <= xb.count * WAVES;
    for (uint32_t base = xb.rank * WAVES; base < nslot; base += xb.count * WAVES) {
        const uint32_t u = base + (uint32_t)w;
        const uint32_t v = spread ? l * nslot + u : u * P + l;
        const bool act = l < (uint32_t)P && u < nslot && v < R.total;
        const int32_t a = region_index_x(R, act ? v : 0);
        int32_t ns1 = 0, s10 = 0;
        if (act) {
            ns1 = E.seg_cnt[a];
            s10 = E.seg_start[a];
            if (ns1 < 0) ns1 = 0;
            if (ns1 > 0) {
                sm.ap[w][l] = E.md_p0[a];
                sm.asv[w][l] = E.md_p2[a].w;
                sm.abar[w][l] = E.md_bar[a] & 1;
            }
            sm.aidx[w][l] = a;
        }
        if (l < (uint32_t)T3_PMAX) sm.cnt[w][l] = 0u;
        const uint32_t incl1 = wave_incl_scan((uint32_t)ns1);
        wave_lds_sync();
        const uint32_t tot = enum_t3(E, K, sm, w, ns1, s10, incl1,
                                     [&](bool ok, int g, int32_t b, int32_t c, float k, uint32_t pos) {
            if (ok) {
                atomicAdd(&sm.cnt[w][g], 1u);
                if (pos < STAGE) {
                    sm.b[w][pos] = b;
                    sm.c[w][pos] = c;
                    sm.k[w][pos] = k;
                    sm.g[w][pos] = (uint8_t)g;
                }
            }
        });
        wave_lds_sync();
        const uint32_t cl = l < (uint32_t)T3_PMAX ? sm.cnt[w][l] : 0u;
        const uint32_t cex = wave_incl_scan(cl) - cl;
        bool ovf;
        const uint32_t off = wave_reserve(tot, E, OT_T3, ovf);
        if (act) {
            E.t3_start[a] = (int32_t)(off + cex);
            E.t3_cnt[a] = ovf ? 0 : (int32_t)cl;
        }
        if (ovf) continue;
        for (uint32_t q = l; q < tot && q < (uint32_t)STAGE; q += 64) {
            E.t3_a[off + q] = sm.aidx[w][sm.g[w][q]];
            E.t3_b[off + q] = sm.b[w][q];
            E.t3_c[off + q] = sm.c[w][q];
            E.t3_k[off + q] = sm.k[w][q];
            E.t3_veto[off + q] = 0;
        }
        if (tot > (uint32_t)STAGE) {
            // beyond the staging: enumerate again and write directly
            enum_t3(E, K, sm, w, ns1, s10, incl1,
                    [&](bool ok, int g, int32_t b, int32_t c, float k, uint32_t pos) {
                if (ok && pos >= STAGE) {
                    E.t3_a[off + pos] = sm.aidx[w][g];
                    E.t3_b[off + pos] = b;
                    E.t3_c[off + pos] = c;
                    E.t3_k[off + pos] = k;
                    E.t3_veto[off + pos] = 0;
                }
            });
        }
        wave_lds_sync();
    }
}

template <int G>
__global__ __launch_bounds__(BLOCK, 6) void k_t3(EvDev E, Consts K)
{
    __shared__ SmT3 sm;
    t3_body<G>(E, K, sm);
}

hipError_t launch_t3(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                     hipStream_t s)
{
    (void)M;
    LST_BY_LANES(lanes, k_t3, dim3(xcd_grid(grid)), dim3(BLOCK), 0, s, E, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- quintuplets
// Candidates of inner MD a: every triplet (a,b,c) followed by every triplet
// (c,d,e).  As for triplets, a wave takes P inner MDs per round (lane l < P
// holds MD l) and walks their first triplets, then the candidates, as one
// list 64 at a time.  sink(ok, g, b, c, d, e, score, pos): g = lane of the
// inner MD, pos = rank among the wave's accepted quintuplets.
template <class F>
__device__ __forceinline__ uint32_t enum_t5(const EvDev &E, const Consts &K, SmT5 &sm,
                                            int w, int32_t nt1, int32_t t10, uint32_t incl1,
                                            F &&sink)
{
    const Grp<64> gw;
    const uint32_t l = (uint32_t)lane_id();
    const unsigned long long below = lanes_below();
    const uint32_t n1 = (uint32_t)__builtin_amdgcn_readlane((int)incl1, 63);
    uint32_t acc = 0;
    for (uint32_t fc = 0; fc < n1; fc += 64) {
        const uint32_t f = fc + l;
        const int g = chunk_src(incl1, (uint32_t)nt1, fc, sm.mark[w]);
        const uint32_t ex1 = gw.bcast(incl1, g) - gw.bcast((uint32_t)nt1, g);
        const int32_t t10g = gw.bcast(t10, g);
        int32_t t1 = 0, cs = 0;
        uint32_t nc = 0;
        if (f < n1) {
            t1 = t10g + (int32_t)(f - ex1);
            const int32_t c = E.t3_c[t1];
            cs = E.t3_start[c];
            nc = (uint32_t)E.t3_cnt[c];
        }
        const uint32_t incl2 = wave_incl_scan(nc);
        const uint32_t n2 = (uint32_t)__builtin_amdgcn_readlane((int)incl2, 63);
        for (uint32_t jc = 0; jc < n2; jc += 64) {
            const uint32_t j = jc + l;
            const int src = chunk_src(incl2, nc, jc, sm.mark[w]);
            const uint32_t ex2 = gw.bcast(incl2, src) - gw.bcast(nc, src);
            const int32_t tt1 = gw.bcast(t1, src), tcs = gw.bcast(cs, src);
            const int gg = gw.bcast(g, src);
            bool ok = false;
            int32_t b = 0, c = 0, d = 0, e = 0;
            float score = 0.0f;
            if (j < n2) {
                const int32_t t2 = tcs + (int32_t)(j - ex2);
                b = E.t3_b[tt1];
                c = E.t3_c[tt1];
                d = E.t3_b[t2];
                e = E.t3_c[t2];
                // a triplet vetoed by the learned scorer joins no quintuplet
                if (!(E.t3_veto[tt1] | E.t3_veto[t2])) {
                    MdV A = {};
                    const float4 ap = sm.ap[w][gg];
                    A.x = ap.x; A.y = ap.y; A.z = ap.z; A.r = ap.w;
                    A.sv = sm.asv[w][gg];
                    A.barrel = sm.abar[w][gg];
                    ok = t5_accept(K, A, load_md(E, b), load_md(E, c), load_md(E, d), load_md(E, e),
                                   E.t3_k[tt1], E.t3_k[t2], score);
                }
            }
            const unsigned long long m = __ballot(ok);
            sink(ok, gg, b, c, d, e, score, acc + (uint32_t)__popcll(m & below));
            acc += (uint32_t)__popcll(m);
        }
    }
    return acc;
}

__device__ __forceinline__ void write_t5(const EvDev &E, uint32_t at, int32_t a, int32_t b,
                                         int32_t c, int32_t d, int32_t e, float score)
{
    E.t5_md0[at] = a;
    E.t5_md1[at] = b;
    E.t5_md2[at] = c;
    E.t5_md3[at] = d;
    E.t5_md4[at] = e;
    E.t5_score[at] = score;
    E.t5_keep[at] = 0;
    E.t5_veto[at] = 0;
}

// G selects P = 256 / G inner MDs per wave and round
template <int G>
__device__ __forceinline__ void t5_body(const EvDev &E, const Consts &K, SmT5 &sm)
{
    if (upstream_overflow(E)) return;
    constexpr int P = 256 / G;
    static_assert(P <= T5_PMAX, "inner MDs per wave");
    const int w = wave_id();
    const uint32_t l = (uint32_t)lane_id();
    const XBlock xb = xcd_block();
    const XRegions R = load_regions_x(E, OT_MD, xb.x);
    // one pass over the sector: lane l of wave slot u takes the u-th MD of the
    // sector's l-th run (as in the segment stage), else consecutive MDs
    const uint32_t nslot = (R.total + P - 1) / P;
    const bool spread = nslot <= xb.count * WAVES;
    for (uint32_t base = xb.rank * WAVES; base < nslot; base += xb.count * WAVES) {
        const uint32_t u = base + (uint32_t)w;
        const uint32_t v = spread ? l * nslot + u : u * P + l;
        const bool act = l < (uint32_t)P && u < nslot && v < R.total;
        const int32_t a = region_index_x(R, act ? v : 0);
        int32_t nt1 = 0, t10 = 0;
        if (act) {
            nt1 = E.t3_cnt[a];
            t10 = E.t3_start[a];
            if (nt1 < 0) nt1 = 0;
            if (nt1 > 0) {
                sm.ap[w][l] = E.md_p0[a];
                sm.asv[w][l] = E.md_p2[a].w;
                sm.abar[w][l] = E.md_bar[a] & 1;
                sm.aidx[w][l] = a;
            }
        }
        const uint32_t incl1 = wave_incl_scan((uint32_t)nt1);
        if (l < (uint32_t)T5_PMAX) sm.cnt[w][l] = 0u;
        wave_lds_sync();
        const uint32_t tot = enum_t5(E, K, sm, w, nt1, t10, incl1,
                                     [&](bool ok, int g, int32_t b, int32_t c, int32_t d,
                                         int32_t e, float sc, uint32_t pos) {
            if (ok) {
                atomicAdd(&sm.cnt[w][g], 1u);
                if (pos < STAGE) {
                    sm.b[w][pos] = b;
                    sm.c[w][pos] = c;
                    sm.d[w][pos] = d;
                    sm.e[w][pos] = e;
                    sm.s[w][pos] = sc;
                    sm.g[w][pos] = (uint8_t)g;
                }
            }
        });
        wave_lds_sync();
        // each inner MD's quintuplets are consecutive, in the list's order
        const uint32_t cl = l < (uint32_t)T5_PMAX ? sm.cnt[w][l] : 0u;
        const uint32_t cex = wave_incl_scan(cl) - cl;
        bool ovf;
        const uint32_t off = wave_reserve(tot, E, OT_T5, ovf);
        if (act) {
            E.t5_start[a] = (int32_t)(off + cex);
            E.t5_cnt[a] = ovf ? 0 : (int32_t)cl;
        }
        if (ovf) continue;
        for (uint32_t q = l; q < tot && q < (uint32_t)STAGE; q += 64)
            write_t5(E, off + q, sm.aidx[w][sm.g[w][q]], sm.b[w][q], sm.c[w][q], sm.d[w][q],
                     sm.e[w][q], sm.s[w][q]);
        if (tot > (uint32_t)STAGE) {
            // beyond the staging: enumerate again and write directly
            enum_t5(E, K, sm, w, nt1, t10, incl1,
                    [&](bool ok, int g, int32_t b, int32_t c, int32_t d, int32_t e, float sc,
                        uint32_t pos) {
                if (ok && pos >= STAGE) write_t5(E, off + pos, sm.aidx[w][g], b, c, d, e, sc);
            });
        }
        wave_lds_sync();
    }
}

template <int G>
__global__ __launch_bounds__(BLOCK, 5) void k_t5(EvDev E, Consts K)
{
    __shared__ SmT5 sm;
    t5_body<G>(E, K, sm);
}

hipError_t launch_t5(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                     hipStream_t s)
{
    (void)M;
    LST_BY_LANES(lanes, k_t5, dim3(xcd_grid(grid)), dim3(BLOCK), 0, s, E, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- duplicate removal
// A quintuplet survives iff for each of its hits it has the smallest key
// (score, hit tuple) among the quintuplets using that hit.  Scores are
// non-negative, so their bit patterns order like the floats.  Quintuplets
// reaching a hit's minimum score are recorded in TIE_SLOTS per-hit slots:
// exact score ties are common (two quintuplets that differ only in the
// upper hit of one mini-doublet have the same anchors, hence the same
// score) and are resolved by the hit tuple.  A quintuplet vetoed by the
// learned scorer takes no part.
//
// one thread per (quintuplet, hit); the hit indices are cached per
// quintuplet ([t][10], sorted and per-event) for the two later passes
__device__ __forceinline__ void dedup_min_body(const EvDev &E, uint32_t *s_pre)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = t5_prefix(E, s_pre) * 10u;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t t = t5_at(E, s_pre, v / 10u);
        const int j = (int)(v % 10u);
        const int32_t h = t5_hit(E, t, j);
        E.t5_hs[(size_t)t * 10 + j] = h;
        E.t5_ho[(size_t)t * 10 + j] = hit_orig(E, h);
        if (E.t5_veto[t]) continue;
        atomicMin(&E.hmin[h], __float_as_uint(E.t5_score[t]));
    }
}

__device__ __forceinline__ void dedup_tie_body(const EvDev &E, uint32_t *s_pre)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = t5_prefix(E, s_pre) * 10u;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t t = t5_at(E, s_pre, v / 10u);
        if (E.t5_veto[t]) continue;
        const int32_t h = E.t5_hs[(size_t)t * 10 + (v % 10u)];
        if (E.hmin[h] == __float_as_uint(E.t5_score[t])) {
            const int k = atomicAdd(&E.htie[h], 1);
            if (k < TIE_SLOTS) {
                E.hslot[(size_t)h * TIE_SLOTS + k] = t;
            } else {
                // further ties: push onto the hit's list in the pool
                const uint32_t s = atomicAdd(&E.gc[GC_TIEPOOL], 1u);
                if (s < E.cap_tpool) {
                    E.tpool_t5[s] = t;
                    E.tpool_next[s] = atomicExch(&E.thead[h], (int32_t)s + 1);
                }
            }
        }
    }
}

// (score-tied) quintuplet u before the one whose per-event hit tuple is `own`
__device__ __forceinline__ bool tuple_less(const EvDev &E, int32_t u, const int32_t *own)
{
    const int2 *p = reinterpret_cast<const int2 *>(E.t5_ho + (size_t)u * 10);
    int32_t o[10];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int2 q = p[k];
        o[2 * k] = q.x;
        o[2 * k + 1] = q.y;
    }
#pragma unroll
    for (int j = 0; j < 10; ++j)
        if (o[j] != own[j]) return o[j] < own[j];
    return false;
}

// one group of 16 lanes per quintuplet: lane j < 10 checks hit j, so the
// ten hits' tie lists are read side by side; the quintuplet is kept iff no
// lane of its group finds a smaller key
constexpr int KEEP_LANES = 16;

__device__ __forceinline__ void dedup_keep_body(const EvDev &E, uint32_t *s_pre)
{
    if (upstream_overflow(E)) return;
    const uint32_t n = t5_prefix(E, s_pre);
    constexpr uint32_t PER_WAVE = 64 / KEEP_LANES, PER_BLOCK = BLOCK / KEEP_LANES;
    const int gl = lane_id() % KEEP_LANES, gi = lane_id() / KEEP_LANES;
    for (uint32_t v0 = blockIdx.x * PER_BLOCK + wave_id() * PER_WAVE; v0 < n;
         v0 += gridDim.x * PER_BLOCK) {
        const uint32_t v = v0 + gi;
        bool bad = false, veto = false;
        int32_t t = 0;
        if (v < n && gl < 10) {
            t = t5_at(E, s_pre, v);
            veto = E.t5_veto[t] != 0;
        }
        if (v < n && gl < 10 && !veto) {
            const float sc = E.t5_score[t];
            const int32_t h = E.t5_hs[(size_t)t * 10 + gl];
            const int nt = E.htie[h];
            bad = E.hmin[h] != __float_as_uint(sc);
            if (!bad && nt > 1) {
                int32_t own[10];
                const int2 *po = reinterpret_cast<const int2 *>(E.t5_ho + (size_t)t * 10);
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const int2 b2 = po[k];
                    own[2 * k] = b2.x;
                    own[2 * k + 1] = b2.y;
                }
                const int ns = nt < TIE_SLOTS ? nt : TIE_SLOTS;
                int32_t us[TIE_SLOTS];
#pragma unroll
                for (int k = 0; k < TIE_SLOTS; ++k)
                    us[k] = k < ns ? E.hslot[(size_t)h * TIE_SLOTS + k] : t;
#pragma unroll
                for (int k = 0; k < TIE_SLOTS; ++k)
                    if (!bad && us[k] != t && tuple_less(E, us[k], own)) bad = true;
                if (!bad && nt > TIE_SLOTS) {
                    // further ties are chained in the pool
                    int listed = 0;
                    for (int32_t e = E.thead[h]; e != 0 && !bad; e = E.tpool_next[e - 1], ++listed) {
                        const int32_t u = E.tpool_t5[e - 1];
                        if (u != t && tuple_less(E, u, own)) bad = true;
                    }
                    if (!bad && listed < nt - TIE_SLOTS) {
                        // the pool ran out: scan every quintuplet (correct, slow)
                        for (uint32_t q = 0; q < n && !bad; ++q) {
                            const int32_t u = t5_at(E, s_pre, q);
                            if (u == t || E.t5_veto[u] || E.t5_score[u] != sc) continue;
                            bool uses = false;
                            for (int k = 0; k < 10; ++k) uses |= (E.t5_hs[(size_t)u * 10 + k] == h);
                            if (uses && tuple_less(E, u, own)) bad = true;
                        }
                    }
                }
            }
        }
        const unsigned long long m = __ballot(bad);
        const bool any_bad = ((m >> (gi * KEEP_LANES)) & ((1ull << KEEP_LANES) - 1ull)) != 0;
        if (v < n && gl == 0) E.t5_keep[t] = (veto || any_bad) ? 0 : 1;
    }
}

__global__ void k_dedup_min(EvDev E)
{
    __shared__ uint32_t s_pre[NSH + 1];
    dedup_min_body(E, s_pre);
}

__global__ void k_dedup_tie(EvDev E)
{
    __shared__ uint32_t s_pre[NSH + 1];
    dedup_tie_body(E, s_pre);
}

__global__ void k_dedup_keep(EvDev E)
{
    __shared__ uint32_t s_pre[NSH + 1];
    dedup_keep_body(E, s_pre);
}

hipError_t launch_dedup(const EvDev &E, const ModDev &M, int grid, hipStream_t s)
{
    (void)M;
    hipLaunchKernelGGL(k_dedup_min, dim3(grid), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_dedup_tie, dim3(grid), dim3(BLOCK), 0, s, E);
    hipLaunchKernelGGL(k_dedup_keep, dim3(grid), dim3(BLOCK), 0, s, E);
    return hipGetLastError();
}

// ---------------------------------------------------------------- scorer features
// the 40 features of every stored quintuplet (one thread each)
__global__ void k_t5_features(EvDev E, Consts K)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n = t5_prefix(E, s_pre);
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t t = t5_at(E, s_pre, v);
        MdV P[5];
        MdX X[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int32_t m = t5_md(E, t, j);
            P[j] = load_md(E, m);
            X[j].bend = E.md_bend[m];
            X[j].is2s = E.md_bar[m] >> 1;
        }
        const float kin = tri_curv(P[0], P[1], P[2]);
        const float kout = tri_curv(P[2], P[3], P[4]);
        float f[40];
        t5_features(K, P, X, kin, kout, f);
        float *out = E.t5_feat + (size_t)t * 40;
#pragma unroll
        for (int j = 0; j < 40; ++j) out[j] = f[j];
    }
}

// the 40 features of every stored triplet (one thread each)
__global__ void k_t3_features(EvDev E, Consts K)
{
    __shared__ uint32_t s_pre[NSH + 1];
    if (upstream_overflow(E)) return;
    const uint32_t n = obj_prefix(E, OT_T3, s_pre);
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t t = obj_at(E, OT_T3, s_pre, v);
        const int32_t m[3] = {E.t3_a[t], E.t3_b[t], E.t3_c[t]};
        MdV P[3];
        MdX X[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            P[j] = load_md(E, m[j]);
            X[j].bend = E.md_bend[m[j]];
            X[j].is2s = E.md_bar[m[j]] >> 1;
        }
        float f[40];
        t3_features(K, P, X, f);
        float *out = E.t3_feat + (size_t)t * 40;
#pragma unroll
        for (int j = 0; j < 40; ++j) out[j] = f[j];
    }
}

hipError_t launch_t3_features(const EvDev &E, const Consts &K, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_t3_features, dim3(grid), dim3(BLOCK), 0, s, E, K);
    return hipGetLastError();
}

hipError_t launch_t5_features(const EvDev &E, const Consts &K, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_t5_features, dim3(grid), dim3(BLOCK), 0, s, E, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------- persistent chain
// All stages in one launch.  Stages are separated by a grid barrier: blocks
// arrive on one of BAR_SH shard counters (blockIdx % BAR_SH); the last block
// of a shard bumps the top counter, which everyone polls.  Release/acquire
// fences at agent scope make one stage's writes visible to every XCD before
// the next stage reads them.  The grid must be co-resident (sized from the
// occupancy query); if it is not, the poll gives up after a bounded time,
// raises error bit 1 and the blocks leave, so the kernel always terminates.
constexpr int BAR_SH = 32;
constexpr int BAR_PAD = 64;   // uint32 stride: each barrier counter on its own 256-byte line
constexpr uint32_t BAR_SPIN_LIMIT = 1u << 19;   // ~0.5 s of polling

__device__ __forceinline__ bool grid_sync(const EvDev &E, uint32_t gen)
{
    __shared__ int s_ok;
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t nsh = G < (uint32_t)BAR_SH ? G : (uint32_t)BAR_SH;
    const uint32_t sh = b % BAR_SH;
    const uint32_t shard_size = (G - sh + BAR_SH - 1) / BAR_SH;
    // the block's stores are complete at the workgroup barrier; one thread
    // then releases them to the device (L2 write-back) and, once everyone has
    // arrived, acquires the others' (invalidation) for the whole block
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t old = atomicAdd(&E.bar[sh * BAR_PAD], 1u);
        if (old + 1u == gen * shard_size) atomicAdd(&E.bar[BAR_SH * BAR_PAD], 1u);
        int ok = 1;
        uint32_t it = 0;
        while (__hip_atomic_load(&E.bar[BAR_SH * BAR_PAD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               gen * nsh) {
            if (++it > BAR_SPIN_LIMIT) {
                ok = 0;
                atomicOr(&E.gc[GC_ERROR], 2u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

__global__ void k_bar_reset(uint32_t *bar)
{
    if (threadIdx.x <= BAR_SH) bar[threadIdx.x * BAR_PAD] = 0u;
}

// G: group width of the four object stages
template <int G>
__global__ __launch_bounds__(BLOCK) void k_chain(EvDev E, ModDev M, Consts K, uint4 *zero_base,
                                                 size_t zero16, int stop)
{
    __shared__ SmChain sm;
    uint32_t gen = 0;
#define LST_SYNC() \
    if (!grid_sync(E, ++gen)) return
    zero_body(zero_base, zero16);
    LST_SYNC();
    hist_body(E, M.n_mod);
    LST_SYNC();
    scan_body(E);
    LST_SYNC();
    scatter_body(E, M);
    LST_SYNC();
    md_body<G>(E, M, K, sm.u.md);
    LST_SYNC();
    seg_body<G, false>(E, M, K, sm.u.seg);
    LST_SYNC();
    t3_body<G>(E, K, sm.u.t3);
    if (stop == PERS_TO_T3) return;
    LST_SYNC();
    t5_body<G>(E, K, sm.u.t5);
    if (stop == PERS_TO_T5) return;
    LST_SYNC();
    dedup_min_body(E, sm.pre);
    LST_SYNC();
    dedup_tie_body(E, sm.pre);
    LST_SYNC();
    dedup_keep_body(E, sm.pre);
#undef LST_SYNC
}

template <int G>
static int occupancy_of_chain()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_chain<G>, BLOCK, 0) != hipSuccess) return 0;
    return nb;
}

int persistent_blocks_per_cu(int lanes)
{
    switch (lanes) {
    case 8: return occupancy_of_chain<8>();
    case 16: return occupancy_of_chain<16>();
    case 32: return occupancy_of_chain<32>();
    default: return occupancy_of_chain<64>();
    }
}

hipError_t launch_chain_persistent(const EvDev &E, const ModDev &M, const Consts &K,
                                   void *zero_base, size_t zero_bytes, int grid, int lanes,
                                   int stop, hipStream_t s)
{
    // whole rounds of sectors (never more blocks than requested: co-residency)
    grid -= grid % NXCD;
    if (grid < NXCD) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, s, E.bar);
    LST_BY_LANES(lanes, k_chain, dim3(grid), dim3(BLOCK), 0, s, E, M, K, (uint4 *)zero_base,
                 zero_bytes / 16, stop);
    return hipGetLastError();
}

}  // namespace lst
