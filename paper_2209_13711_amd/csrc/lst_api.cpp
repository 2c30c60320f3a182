// Host side of liblst: the C ABI declared in include/lst.h.
//
// Owns the geometry on the device, carves the per-batch arrays out of the
// caller's arena, enqueues the stage kernels on the caller's stream and
// converts device objects into per-event hit-index tuples on request.
#include "../../include/lst.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lst_internal.hpp"

namespace lst {
void build_module_map(int n, const float *f32, const int32_t *i32, const double *params,
                      std::vector<int32_t> &row_ptr, std::vector<int32_t> &col);
}

using namespace lst;

struct lst_ctx {
    int device = 0;
    double params[LST_N_PARAMS];
    Consts K;
    std::string err;
    // geometry
    int n_mod = 0;
    std::vector<float> mod_f32;
    std::vector<int32_t> mod_i32;
    std::vector<int32_t> map_ptr, map_col;
    void *geo_dev = nullptr;
    ModDev M{};
    // arena
    char *arena = nullptr;
    size_t arena_bytes = 0;
    lst_caps caps{};
    EvDev E{};
    void *zero_base = nullptr;
    size_t zero_bytes = 0;
    // batch
    int n_events = 0;
    std::vector<int32_t> hit_off;
    // pinned staging: batch descriptor, hit offsets, then (host inputs) x, y,
    // z, module, sensor, so that every upload is a DMA from pinned memory
    int32_t *stage_host = nullptr;
    size_t stage_cap = 0;   // bytes
    hipEvent_t stage_done = nullptr;
    bool stage_pending = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    Tuning tune{};
    int n_cu = 0;
    bool features_valid = false;
    // learned scorer
    int mode = LST_MODE_CUTS;
    // per kind (0 triplets, 1 quintuplets): params [MLP_NPARAM], mean [40], istd [40]
    float *mlp_dev[2] = {nullptr, nullptr};
    float mlp_threshold[2] = {0.0f, 0.0f};
    bool fallback = false;   // the running batch: scorer mode without a network
    bool t3_features_valid = false;
    void *fixed_work = nullptr;   // this device's copy of the fixed backward workspace
    int32_t cap[OT_COUNT] = {0, 0, 0, 0};   // per-module capacities (0: none)
    int32_t half16 = 0;                       // half-precision hit storage
    // pixel objects: constants of the loaded pixel parameters, host copy of
    // the batch's seed and pixel offsets, loaded for the current hits
    PixConsts pxk{};
    std::vector<int32_t> px_off, sd_off;
    bool px_loaded = false;
    std::vector<lst_counts> counts;
    bool counts_valid = false;
    int stage = 0;  // 0 nothing, 1 hits loaded, 2 sorted, 3 md, 4 seg, 5 t3, 6 t5, 7 dedup
    bool sort_ev_ok = false;   // the per-event LDS sort can run on this geometry
};

static int fail(lst_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(c, call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) return fail((c), LST_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// FP32 constants, each computed once in FP64 from the primary parameters and
// rounded once.
static void derive(const double *p, Consts &K)
{
    const double kmax = (0.0029979245800 * p[LST_P_BFIELD]) / p[LST_P_PTMIN];
    const double klim = kmax * (1.0 + p[LST_P_EPSK]);
    K.kmax = (float)kmax;
    K.klim = (float)klim;
    K.kh = (float)(0.5 * klim);
    K.tolu = (float)(p[LST_P_NSIG] * std::sqrt(2.0) * p[LST_P_SIGU]);
    K.tolv = (float)(p[LST_P_NSIG] * std::sqrt(2.0) * p[LST_P_SIGV]);
    K.tolkc = (float)(p[LST_P_NSIG] * 8.0 * std::sqrt(1.5));
    K.epsak = (float)(p[LST_P_EPSA] * kmax);
    K.z0max = (float)p[LST_P_Z0MAX];
    K.sigu = (float)p[LST_P_SIGU];
    K.sigv = (float)p[LST_P_SIGV];
    K.nsig = (float)p[LST_P_NSIG];
    K.d0max = (float)p[LST_P_D0MAX];
    K.w = (float)p[LST_P_W];
    K.w2 = (float)(p[LST_P_W] * p[LST_P_W]);
    K.xrphi = (float)p[LST_P_XRPHI];
    K.xrz = (float)p[LST_P_XRZ];
}

// ---------------------------------------------------------------- arena
namespace {
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(char *b) : base(b) {}
    template <class T>
    T *take(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += sizeof(T) * std::max<size_t>(n, 1);
        return p;
    }
};

bool caps_ok(const lst_caps *k)
{
    return k && k->events > 0 && k->hits >= 0 && k->md >= 0 && k->seg >= 0 && k->t3 >= 0 &&
           k->t5 >= 0 && k->hits < (1ll << 31) && k->md < (1ll << 31) &&
           k->seg < (1ll << 31) && k->t3 < (1ll << 31) && k->t5 < (1ll << 31) &&
           k->px_hits >= 0 && k->seeds >= 0 && k->px_cand >= 0 && k->px_hits < (1ll << 31) &&
           k->seeds < (1ll << 29) && k->px_cand < (1ll << 31);
}

// Lay the arrays out; with base == nullptr only the size is computed.
size_t carve(lst_ctx *c, char *base, const lst_caps &k, EvDev &E, void **zero_base,
             size_t *zero_bytes)
{
    Carver cv(base);
    const int64_t slots = (int64_t)k.events * c->n_mod;
    const int64_t keys = 2 * slots;
    E = EvDev{};
    E.cap_ev = k.events;
    E.cap_slots = (int32_t)slots;
    E.cap_keys = (int32_t)keys;
    E.desc = cv.take<int32_t>(D_COUNT);
    E.bar = cv.take<uint32_t>(33 * 64);   // 33 barrier counters, one 256-byte line each
    E.cap_hits = k.hits;
    const int64_t caps[OT_COUNT] = {k.md, k.seg, k.t3, k.t5};
    size_t span[OT_COUNT];
    for (int t = 0; t < OT_COUNT; ++t) {
        E.rc[t] = (uint32_t)std::max<int64_t>(1, (caps[t] + NSH - 1) / NSH);
        span[t] = (size_t)E.rc[t] * NSH;
    }
    const size_t nmd = span[OT_MD], nseg = span[OT_SEG], nt3 = span[OT_T3], nt5 = span[OT_T5];
    // region cleared at the start of every chain
    size_t z0 = (cv.off + 255) & ~(size_t)255;
    E.gc = cv.take<uint32_t>(GC_COUNT);
    E.bcnt = cv.take<uint32_t>(keys);
    E.scan_st = cv.take<unsigned long long>((keys + 1 + SCAN_TILE - 1) / SCAN_TILE);
    size_t z1 = (cv.off + 255) & ~(size_t)255;
    if (zero_base) *zero_base = base ? base + z0 : nullptr;
    if (zero_bytes) *zero_bytes = z1 - z0;
    // inputs
    E.x = cv.take<float>(k.hits);
    E.y = cv.take<float>(k.hits);
    E.z = cv.take<float>(k.hits);
    E.module = cv.take<int32_t>(k.hits);
    E.sensor = cv.take<uint8_t>(k.hits);
    E.hit_off = cv.take<int32_t>(k.events + 1);
    // grouping
    E.hrank = cv.take<uint32_t>(k.hits);
    E.boff = cv.take<uint32_t>(keys + 1);
    E.hsort = cv.take<float4>(k.hits);
    E.hsort_h = cv.take<uint2>(k.hits);
    E.hmin = cv.take<uint32_t>(k.hits);
    E.htie = cv.take<int32_t>(k.hits);
    E.hslot = cv.take<int32_t>((size_t)k.hits * TIE_SLOTS);
    E.thead = cv.take<int32_t>(k.hits);
    E.cap_tpool = (uint32_t)std::max<int64_t>(4096, k.t5 / 8);
    E.tpool_t5 = cv.take<int32_t>(E.cap_tpool);
    E.tpool_next = cv.take<int32_t>(E.cap_tpool);
    // MD
    E.md_hlo = cv.take<int32_t>(nmd);
    E.md_hup = cv.take<int32_t>(nmd);
    E.md_slot = cv.take<int32_t>(nmd);
    E.md_nbr = cv.take<int4>(nmd);
    E.md_p0 = cv.take<float4>(nmd);
    E.md_p1 = cv.take<float4>(nmd);
    E.md_p2 = cv.take<float4>(nmd);
    E.md_bend = cv.take<float>(nmd);
    E.md_atol = cv.take<float>(nmd);

    E.md_bar = cv.take<uint8_t>(nmd);
    E.md_start = cv.take<int32_t>(slots);
    E.md_cnt = cv.take<int32_t>(slots);
    // segments
    E.seg_in = cv.take<int32_t>(nseg);
    E.seg_out = cv.take<int32_t>(nseg);
    E.seg_start = cv.take<int32_t>(nmd);
    E.seg_cnt = cv.take<int32_t>(nmd);
    // triplets
    E.t3_a = cv.take<int32_t>(nt3);
    E.t3_b = cv.take<int32_t>(nt3);
    E.t3_c = cv.take<int32_t>(nt3);
    E.t3_k = cv.take<float>(nt3);
    E.t3_start = cv.take<int32_t>(nmd);
    E.t3_cnt = cv.take<int32_t>(nmd);
    E.t3_veto = cv.take<uint8_t>(nt3);
    E.t3_logit = cv.take<float>(nt3);
    E.t3_feat = k.features ? cv.take<float>(nt3 * 40) : nullptr;
    // quintuplets
    E.t5_md0 = cv.take<int32_t>(nt5);
    E.t5_md1 = cv.take<int32_t>(nt5);
    E.t5_md2 = cv.take<int32_t>(nt5);
    E.t5_md3 = cv.take<int32_t>(nt5);
    E.t5_md4 = cv.take<int32_t>(nt5);
    E.t5_score = cv.take<float>(nt5);
    E.t5_keep = cv.take<uint8_t>(nt5);
    E.t5_veto = cv.take<uint8_t>(nt5);
    E.t5_hs = cv.take<int32_t>(nt5 * 10);
    E.t5_ho = cv.take<int32_t>(nt5 * 10);
    E.t5_feat = k.features ? cv.take<float>(nt5 * 40) : nullptr;
    E.t5_logit = cv.take<float>(nt5);
    E.t5_start = cv.take<int32_t>(nmd);
    E.t5_cnt = cv.take<int32_t>(nmd);
    // per-module capacities
    const size_t span_max = std::max(std::max(nmd, nseg), std::max(nt3, nt5));
    uint32_t rc_max = 0;
    for (int t = 0; t < OT_COUNT; ++t) rc_max = std::max(rc_max, E.rc[t]);
    E.cap_drop = cv.take<uint8_t>((span_max + 15) & ~(size_t)15);
    E.cap_pre = cv.take<int32_t>((size_t)NSH * (rc_max + 1));
    E.cap_nd = cv.take<uint32_t>(((size_t)k.events * OT_COUNT + 3) & ~(size_t)3);
    // pixel objects (only with pixel capacities)
    E.cap_px = (int32_t)k.px_hits;
    E.cap_seeds = (int32_t)k.seeds;
    E.cap_pxc = (int32_t)k.px_cand;
    if (k.seeds > 0) {
        E.px_x = cv.take<float>(k.px_hits);
        E.px_y = cv.take<float>(k.px_hits);
        E.px_z = cv.take<float>(k.px_hits);
        E.px_off = cv.take<int32_t>(k.events + 1);
        E.sd_off = cv.take<int32_t>(k.events + 1);
        E.sd_hits = cv.take<int32_t>((size_t)k.seeds * 4);
        E.sd_ev = cv.take<int32_t>(k.seeds);
        E.sd_local = cv.take<int32_t>(k.seeds);
        E.sd_dir = cv.take<float4>(k.seeds);
        E.sd_used = cv.take<uint8_t>(k.seeds);
        E.sd_keep = cv.take<uint8_t>(k.seeds);
        E.t5_dir = cv.take<float4>(nt5);
        E.t3_dir = cv.take<float4>(nt3);
        E.t5_clean = cv.take<uint8_t>(nt5);
        const size_t pl_n = (size_t)PXL_COUNT * ((size_t)k.events * PX_NB + 1);
        E.pl_cnt = cv.take<int32_t>(pl_n);
        E.pl_fill = cv.take<int32_t>(pl_n);
        E.pl_off = cv.take<int32_t>(pl_n);
        E.pl_k5 = cv.take<int32_t>(nt5);
        E.pl_k3 = cv.take<int32_t>(nt3);
        E.pl_k5d = cv.take<float4>(nt5);
        E.pl_k3d = cv.take<float4>(nt3);
        E.pl_d5 = cv.take<float4>(k.px_cand);
        E.pl_d3 = cv.take<float4>(k.px_cand);
        E.pl_dt = cv.take<float4>(nt5);
        E.c5_seed = cv.take<int32_t>(k.px_cand);
        E.c5_obj = cv.take<int32_t>(k.px_cand);
        E.c5_score = cv.take<float>(k.px_cand);
        E.c5_keep = cv.take<uint8_t>(k.px_cand);
        E.c3_seed = cv.take<int32_t>(k.px_cand);
        E.c3_obj = cv.take<int32_t>(k.px_cand);
        E.c3_score = cv.take<float>(k.px_cand);
        E.c3_keep = cv.take<uint8_t>(k.px_cand);
        E.sd_c5 = cv.take<int2>(k.seeds);
        E.sd_c3 = cv.take<int2>(k.seeds);
        E.sd_free = cv.take<int32_t>(k.seeds);
        E.hmin_o = cv.take<unsigned long long>(k.hits);
        E.hmin_p = cv.take<unsigned long long>(k.px_hits);
        E.hflag_o = cv.take<uint8_t>(k.hits);
        E.hflag_p = cv.take<uint8_t>(k.px_hits);
    }
    return (cv.off + 255) & ~(size_t)255;
}
}  // namespace

template <class T>
static int d2h(lst_ctx *c, std::vector<T> &v, const T *src, size_t n)
{
    v.resize(std::max<size_t>(n, 1));
    if (n) HIPCHK(c, hipMemcpy(v.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost));
    return LST_OK;
}

// per-event index of each of the first n sorted hits
static int sorted_orig(lst_ctx *c, std::vector<int32_t> &out, size_t n)
{
    out.resize(std::max<size_t>(n, 1));
    if (c->E.half16) {
        std::vector<uint2> h;
        int rc = d2h(c, h, (const uint2 *)c->E.hsort_h, n);
        if (rc) return rc;
        for (size_t i = 0; i < n; ++i) out[i] = (int32_t)h[i].y;
        return LST_OK;
    }
    std::vector<float4> h;
    int rc = d2h(c, h, (const float4 *)c->E.hsort, n);
    if (rc) return rc;
    for (size_t i = 0; i < n; ++i) std::memcpy(&out[i], &h[i].w, sizeof(int32_t));
    return LST_OK;
}

// pinned staging layout: [descriptor][offsets] then the host hit arrays
static size_t stage_hits_offset(int64_t events)
{
    return ((sizeof(int32_t) * ((size_t)events + 1 + D_COUNT)) + 255) & ~(size_t)255;
}

static size_t stage_bytes(int64_t events, int64_t hits)
{
    return stage_hits_offset(events) + (size_t)hits * (3 * sizeof(float) + sizeof(int32_t) + 1);
}

extern "C" {

int lst_create(lst_ctx **out, int device, const double *params, int32_t n_params)
{
    if (!out) return LST_E_INVALID;
    *out = nullptr;
    if (!params || n_params < LST_N_PARAMS) return LST_E_INVALID;
    for (int i = 0; i < LST_N_PARAMS; ++i)
        if (!std::isfinite(params[i])) return LST_E_INVALID;
    if (params[LST_P_BFIELD] <= 0 || params[LST_P_PTMIN] <= 0 || params[LST_P_W] <= 0)
        return LST_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return LST_E_HIP;
    // device address of the fixed backward workspace on this GPU (lst_mlp_backward_noalloc)
    void *fixed = nullptr;
    if (mlp_fixed_scratch(device, &fixed) != hipSuccess || !fixed) return LST_E_HIP;
    lst_ctx *c = new (std::nothrow) lst_ctx();
    if (!c) return LST_E_NOMEM;
    c->device = device;
    c->fixed_work = fixed;
    std::memcpy(c->params, params, sizeof(c->params));
    derive(c->params, c->K);
    *out = c;
    return LST_OK;
}

static void drop_graph(lst_ctx *c)
{
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

void lst_destroy(lst_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    drop_graph(c);
    if (c->stage_done) (void)hipEventSynchronize(c->stage_done);
    if (c->stage_done) (void)hipEventDestroy(c->stage_done);
    if (c->stage_host) (void)hipHostFree(c->stage_host);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->geo_dev) (void)hipFree(c->geo_dev);
    for (float *p : c->mlp_dev)
        if (p) (void)hipFree(p);
    delete c;
}

const char *lst_last_error(const lst_ctx *c) { return c ? c->err.c_str() : "no context"; }

int lst_load_geometry(lst_ctx *c, int32_t n, const float *f32, const int32_t *i32)
{
    if (!c) return LST_E_INVALID;
    if (n <= 0 || !f32 || !i32) return fail(c, LST_E_INVALID, "empty geometry");
    for (int m = 0; m < n; ++m) {
        int layer = i32[m], sub = i32[n + m];
        if (layer < 1 || layer > 16 || sub < 0 || sub > 1)
            return fail(c, LST_E_INVALID, "module %d: bad layer/subdetector", m);
        for (int f = 0; f < LST_MOD_NF; ++f)
            if (!std::isfinite(f32[(size_t)f * n + m]))
                return fail(c, LST_E_INVALID, "module %d: non-finite field %d", m, f);
    }
    HIPCHK(c, hipSetDevice(c->device));
    c->n_mod = n;
    c->mod_f32.assign(f32, f32 + (size_t)LST_MOD_NF * n);
    c->mod_i32.assign(i32, i32 + (size_t)LST_MOD_NI * n);
    build_module_map(n, f32, i32, c->params, c->map_ptr, c->map_col);

    // device geometry: 14 float rows, barrel flags, map
    std::vector<float> rows((size_t)14 * n);
    std::vector<int32_t> barrel(2 * (size_t)n);   // barrel flags, then 2S flags
    const int src[10] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 14};  // cx..vz, gap
    for (int r = 0; r < 10; ++r)
        std::memcpy(&rows[(size_t)r * n], &f32[(size_t)src[r] * n], sizeof(float) * n);
    for (int m = 0; m < n; ++m) {
        const float cx = f32[m], cy = f32[n + m], wx = f32[9 * n + m], wy = f32[10 * n + m];
        const float g = f32[14 * n + m];
        rows[(size_t)10 * n + m] = ((cx * wx) + (cy * wy)) - (0.5f * g);  // lower-sensor apothem
        rows[(size_t)11 * n + m] = wx;                                     // sensor normal
        rows[(size_t)12 * n + m] = wy;
        rows[(size_t)13 * n + m] = f32[11 * n + m];
        barrel[m] = i32[n + m] == 0 ? 1 : 0;
        barrel[(size_t)n + m] = i32[3 * n + m] == 1 ? 1 : 0;
    }
    const size_t nf = rows.size() * sizeof(float);
    const size_t nb = sizeof(int32_t) * 2 * n;
    const size_t np = sizeof(int32_t) * (n + 1);
    const size_t nc = sizeof(int32_t) * std::max<size_t>(c->map_col.size(), 1);
    // modules by azimuthal sector (NXCD sectors of the module centre's phi), then layer
    std::vector<int32_t> order(n), sector(n);
    int32_t sec_cnt[NXCD] = {};
    for (int m = 0; m < n; ++m) {
        const double phi = std::atan2((double)f32[n + m], (double)f32[m]);   // (-pi, pi]
        int s = (int)std::floor((phi + M_PI) / (2.0 * M_PI) * NXCD);
        sector[m] = std::min(NXCD - 1, std::max(0, s));
        ++sec_cnt[sector[m]];
        order[m] = m;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (sector[a] != sector[b]) return sector[a] < sector[b];
        return i32[a] < i32[b];   // layer
    });
    const size_t no = sizeof(int32_t) * n;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t total = al(nf) + al(nb) + al(np) + al(nc) + al(no);
    if (c->geo_dev) {
        HIPCHK(c, hipFree(c->geo_dev));
        c->geo_dev = nullptr;
    }
    HIPCHK(c, hipMalloc(&c->geo_dev, total));
    char *p = (char *)c->geo_dev;
    float *drows = (float *)p;
    int32_t *dbar = (int32_t *)(p + al(nf));
    int32_t *dptr = (int32_t *)(p + al(nf) + al(nb));
    int32_t *dcol = (int32_t *)(p + al(nf) + al(nb) + al(np));
    int32_t *dord = (int32_t *)(p + al(nf) + al(nb) + al(np) + al(nc));
    HIPCHK(c, hipMemcpy(dord, order.data(), no, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(drows, rows.data(), nf, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(dbar, barrel.data(), nb, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(dptr, c->map_ptr.data(), np, hipMemcpyHostToDevice));
    if (!c->map_col.empty())
        HIPCHK(c, hipMemcpy(dcol, c->map_col.data(), c->map_col.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice));
    ModDev &M = c->M;
    float *r[14];
    for (int i = 0; i < 14; ++i) r[i] = drows + (size_t)i * n;
    M.cx = r[0]; M.cy = r[1]; M.cz = r[2]; M.ux = r[3]; M.uy = r[4]; M.uz = r[5];
    M.vx = r[6]; M.vy = r[7]; M.vz = r[8]; M.g = r[9]; M.rl = r[10];
    M.wx = r[11]; M.wy = r[12]; M.wz = r[13];
    M.barrel = dbar;
    M.is2s = dbar + n;
    M.map_ptr = dptr;
    M.map_col = dcol;
    M.xorder = dord;
    M.sec_off[0] = 0;
    for (int x = 0; x < NXCD; ++x) M.sec_off[x + 1] = M.sec_off[x] + sec_cnt[x];
    M.n_mod = n;
    // batches sort each event's hits in LDS when its bins fit there
    c->sort_ev_ok = sort_ev_lds_bytes(n) <= SORT_EV_LDS_MAX && sort_ev_prepare(n) == hipSuccess;
    (void)hipGetLastError();
    c->arena = nullptr;  // a new geometry invalidates the arena layout
    drop_graph(c);
    c->stage = 0;
    return LST_OK;
}

// the per-event sort for batches of at least SORT_EV_MIN_EVENTS events
static bool sort_per_event(const lst_ctx *c)
{
    return c->sort_ev_ok && c->caps.events >= SORT_EV_MIN_EVENTS;
}

// the segment kernel whose runs of inner MDs of one module share their
// candidate enumeration, for arenas that hold more than one event (a wave
// then takes consecutive MDs); one event spreads its MDs over the waves
static bool seg_share(const lst_ctx *c) { return c->caps.events > 1; }

int lst_build_map(const double *params, int32_t n_params, int32_t n, const float *f32,
                  const int32_t *i32, int32_t *row_ptr, int32_t *col, int64_t cap_col,
                  int64_t *n_edges)
{
    if (!params || n_params < LST_N_PARAMS || n <= 0 || !f32 || !i32) return LST_E_INVALID;
    std::vector<int32_t> ptr, cl;
    build_module_map(n, f32, i32, params, ptr, cl);
    if (n_edges) *n_edges = (int64_t)cl.size();
    if (row_ptr) std::memcpy(row_ptr, ptr.data(), sizeof(int32_t) * (n + 1));
    if ((int64_t)cl.size() > cap_col) return LST_E_CAPACITY;
    if (col && !cl.empty()) std::memcpy(col, cl.data(), sizeof(int32_t) * cl.size());
    return LST_OK;
}

int lst_get_map(lst_ctx *c, int32_t *row_ptr, int32_t *col, int64_t cap_col, int64_t *n_edges)
{
    if (!c) return LST_E_INVALID;
    if (!c->n_mod) return fail(c, LST_E_STATE, "no geometry loaded");
    if (n_edges) *n_edges = (int64_t)c->map_col.size();
    if (row_ptr) std::memcpy(row_ptr, c->map_ptr.data(), sizeof(int32_t) * (c->n_mod + 1));
    if ((int64_t)c->map_col.size() > cap_col)
        return fail(c, LST_E_CAPACITY, "map has %zu edges", c->map_col.size());
    if (col && !c->map_col.empty())
        std::memcpy(col, c->map_col.data(), sizeof(int32_t) * c->map_col.size());
    return LST_OK;
}

// ---------------------------------------------------------------- arena

static int clamp_grid(int64_t g) { return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65535)); }

// Launch shapes before tuning: one wave per work item up to 2048 blocks.
// launch shape before tuning: the best measured on a PU200-like event
static void default_tuning(lst_ctx *c)
{
    Tuning &t = c->tune;
    t.grid[ST_SORT] = clamp_grid(std::min<int64_t>((c->caps.hits + BLOCK - 1) / BLOCK, GRID_MAX));
    t.grid[ST_MD] = GRID_MAX;
    t.grid[ST_SEG] = 2 * GRID_MAX;
    t.grid[ST_T3] = GRID_MAX;
    t.grid[ST_T5] = 2 * GRID_MAX;
    t.grid[ST_DEDUP] = 1024;
    for (int i = 0; i < ST_COUNT; ++i) t.lanes[i] = 64;
    t.lanes[ST_MD] = 32;
    t.lanes[ST_SEG] = 32;
    t.lanes[ST_T3] = 32;
    t.lanes[ST_T5] = 16;
    t.persistent = 0;
    t.blocks_per_cu = std::max(1, std::min(2, persistent_blocks_per_cu(t.lanes[ST_SEG])));
}

int lst_arena_bytes(const lst_ctx *cc, const lst_caps *caps, size_t *bytes)
{
    lst_ctx *c = const_cast<lst_ctx *>(cc);
    if (!c || !bytes) return LST_E_INVALID;
    if (!c->n_mod) return fail(c, LST_E_STATE, "no geometry loaded");
    if (!caps_ok(caps)) return fail(c, LST_E_INVALID, "bad capacities");
    if ((int64_t)caps->events * c->n_mod * 2 >= (1ll << 31))
        return fail(c, LST_E_INVALID, "too many events for one arena");
    EvDev E;
    *bytes = carve(c, nullptr, *caps, E, nullptr, nullptr);
    return LST_OK;
}

int lst_attach_arena(lst_ctx *c, void *dev_ptr, size_t bytes, const lst_caps *caps)
{
    if (!c) return LST_E_INVALID;
    size_t need = 0;
    int rc = lst_arena_bytes(c, caps, &need);
    if (rc != LST_OK) return rc;
    if (!dev_ptr) return fail(c, LST_E_INVALID, "null arena");
    if (((uintptr_t)dev_ptr & 255) != 0) return fail(c, LST_E_INVALID, "arena not 256-byte aligned");
    if (bytes < need) return fail(c, LST_E_CAPACITY, "arena needs %zu bytes, got %zu", need, bytes);
    HIPCHK(c, hipSetDevice(c->device));
    drop_graph(c);
    if (c->stage_pending) {
        HIPCHK(c, hipEventSynchronize(c->stage_done));
        c->stage_pending = false;
    }
    const size_t want = stage_bytes(caps->events, caps->hits);
    if (c->stage_cap < want) {
        if (c->stage_host) HIPCHK(c, hipHostFree(c->stage_host));
        c->stage_host = nullptr;
        HIPCHK(c, hipHostMalloc((void **)&c->stage_host, want, hipHostMallocDefault));
        c->stage_cap = want;
    }
    if (!c->stage_done) HIPCHK(c, hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming));
    c->arena = (char *)dev_ptr;
    c->arena_bytes = bytes;
    c->caps = *caps;
    carve(c, c->arena, *caps, c->E, &c->zero_base, &c->zero_bytes);
    c->E.half16 = c->half16;
    // bin counts start at zero (each sort leaves them at zero again)
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, launch_zero(c->E, c->zero_base, c->zero_bytes, nullptr));
    // capacity drop flags start at zero (each compaction leaves them at zero)
    {
        const size_t span_max = std::max(std::max(c->E.rc[OT_MD], c->E.rc[OT_SEG]),
                                         std::max(c->E.rc[OT_T3], c->E.rc[OT_T5])) * (size_t)NSH;
        HIPCHK(c, launch_zero(c->E, c->E.cap_drop, (span_max + 15) & ~(size_t)15, nullptr));
    }
    HIPCHK(c, hipDeviceSynchronize());
    if (!c->n_cu) HIPCHK(c, hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    default_tuning(c);
    c->stage = 0;
    c->n_events = 0;
    return LST_OK;
}

int lst_load_hits(lst_ctx *c, int32_t n_events, const int32_t *hit_offsets, const float *x,
                  const float *y, const float *z, const int32_t *module, const uint8_t *sensor,
                  int on_device, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (!c->n_mod) return fail(c, LST_E_STATE, "no geometry loaded");
    if (!c->arena) return fail(c, LST_E_STATE, "no arena attached");
    if (n_events <= 0 || n_events > c->caps.events || !hit_offsets)
        return fail(c, LST_E_INVALID, "n_events %d outside 1..%d", n_events, c->caps.events);
    if (hit_offsets[0] != 0) return fail(c, LST_E_INVALID, "hit_offsets[0] must be 0");
    for (int e = 0; e < n_events; ++e)
        if (hit_offsets[e + 1] < hit_offsets[e]) return fail(c, LST_E_INVALID, "hit_offsets not sorted");
    const int64_t n = hit_offsets[n_events];
    if (n > c->caps.hits) return fail(c, LST_E_CAPACITY, "%lld hits exceed capacity %lld",
                                      (long long)n, (long long)c->caps.hits);
    if (n > 0 && (!x || !y || !z || !module || !sensor))
        return fail(c, LST_E_INVALID, "null hit array");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    EvDev &E = c->E;
    // the pinned buffer is reused: wait until the previous batch's copies have left it
    if (c->stage_pending) HIPCHK(c, hipEventSynchronize(c->stage_done));
    if (n > 0 && on_device) {
        HIPCHK(c, hipMemcpyAsync(E.x, x, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.y, y, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.z, z, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.module, module, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.sensor, sensor, n, hipMemcpyDeviceToDevice, s));
    } else if (n > 0) {
        // host arrays: one host copy into pinned memory, then DMA (a copy from
        // pageable memory goes through the runtime's own staging, several
        // times slower)
        char *hp = (char *)c->stage_host + stage_hits_offset(c->caps.events);
        const size_t nb = sizeof(float) * n;
        char *px = hp, *py = px + nb, *pz = py + nb, *pm = pz + nb, *ps = pm + nb;
        std::memcpy(px, x, nb);
        std::memcpy(py, y, nb);
        std::memcpy(pz, z, nb);
        std::memcpy(pm, module, sizeof(int32_t) * n);
        std::memcpy(ps, sensor, n);
        HIPCHK(c, hipMemcpyAsync(E.x, px, nb, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.y, py, nb, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.z, pz, nb, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.module, pm, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(E.sensor, ps, n, hipMemcpyHostToDevice, s));
    }
    c->hit_off.assign(hit_offsets, hit_offsets + n_events + 1);
    int32_t *st = c->stage_host;
    st[D_NEV] = n_events;
    st[D_NHITS] = (int32_t)n;
    st[D_NSLOTS] = n_events * c->n_mod;
    st[D_NKEYS] = 2 * n_events * c->n_mod;
    st[D_NPX] = 0;      // pixel objects belong to one batch: load them after the hits
    st[D_NSEEDS] = 0;
    c->px_loaded = false;
    std::memcpy(st + D_COUNT, hit_offsets, sizeof(int32_t) * (n_events + 1));
    HIPCHK(c, hipMemcpyAsync((void *)E.desc, st, sizeof(int32_t) * D_COUNT, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(E.hit_off, st + D_COUNT, sizeof(int32_t) * (n_events + 1),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipEventRecord(c->stage_done, s));
    c->stage_pending = true;
    c->n_events = n_events;
    c->stage = 1;
    return LST_OK;
}

int lst_load_pixel(lst_ctx *c, int32_t n_events, const int32_t *px_offsets, const float *x,
                   const float *y, const float *z, const int32_t *seed_offsets,
                   const int32_t *seeds, const double *pp, int32_t n_pp, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (c->stage < 1) return fail(c, LST_E_STATE, "load the hits of the batch first");
    if (n_events != c->n_events || !px_offsets || !seed_offsets)
        return fail(c, LST_E_INVALID, "pixel batch of %d events, hits of %d", n_events, c->n_events);
    if (c->caps.seeds < 1 || c->caps.px_cand < 1 || !c->E.sd_hits)
        return fail(c, LST_E_CAPACITY, "the arena holds no pixel objects (caps.seeds, caps.px_cand)");
    if (!pp || n_pp < LST_PX_N_PARAMS) return fail(c, LST_E_INVALID, "pixel parameters");
    for (int i = 0; i < LST_PX_N_PARAMS; ++i)
        if (!std::isfinite(pp[i]) || pp[i] < 0) return fail(c, LST_E_INVALID, "pixel parameter %d", i);
    if (px_offsets[0] != 0 || seed_offsets[0] != 0)
        return fail(c, LST_E_INVALID, "pixel and seed offsets start at 0");
    for (int e = 0; e < n_events; ++e)
        if (px_offsets[e + 1] < px_offsets[e] || seed_offsets[e + 1] < seed_offsets[e])
            return fail(c, LST_E_INVALID, "pixel or seed offsets not sorted");
    const int64_t n_px = px_offsets[n_events], n_sd = seed_offsets[n_events];
    if (n_px > c->caps.px_hits || n_sd > c->caps.seeds)
        return fail(c, LST_E_CAPACITY, "%lld pixel hits and %lld seeds exceed capacities %lld, %lld",
                    (long long)n_px, (long long)n_sd, (long long)c->caps.px_hits,
                    (long long)c->caps.seeds);
    if ((n_px > 0 && (!x || !y || !z)) || (n_sd > 0 && !seeds))
        return fail(c, LST_E_INVALID, "null pixel array");
    std::vector<int32_t> hits((size_t)n_sd * 4), ev((size_t)n_sd), loc((size_t)n_sd);
    for (int e = 0; e < n_events; ++e)
        for (int32_t q = seed_offsets[e]; q < seed_offsets[e + 1]; ++q) {
            const int32_t n_e = px_offsets[e + 1] - px_offsets[e];
            for (int k = 0; k < 4; ++k) {
                const int32_t h = seeds[4 * (size_t)q + k];
                if (h < 0 || h >= n_e)
                    return fail(c, LST_E_INVALID, "seed %d of event %d: pixel hit %d outside 0..%d",
                                q - seed_offsets[e], e, h, n_e - 1);
                hits[4 * (size_t)q + k] = px_offsets[e] + h;
            }
            ev[q] = e;
            loc[q] = q - seed_offsets[e];
        }
    HIPCHK(c, hipSetDevice(c->device));
    // the stream may still read the previous pixel batch: copy after it
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    const EvDev &E = c->E;
    if (n_px > 0) {
        HIPCHK(c, hipMemcpy(E.px_x, x, sizeof(float) * n_px, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(E.px_y, y, sizeof(float) * n_px, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(E.px_z, z, sizeof(float) * n_px, hipMemcpyHostToDevice));
    }
    if (n_sd > 0) {
        HIPCHK(c, hipMemcpy(E.sd_hits, hits.data(), sizeof(int32_t) * hits.size(), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(E.sd_ev, ev.data(), sizeof(int32_t) * ev.size(), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(E.sd_local, loc.data(), sizeof(int32_t) * loc.size(), hipMemcpyHostToDevice));
    }
    if (E.px_off) {
        HIPCHK(c, hipMemcpy(E.px_off, px_offsets, sizeof(int32_t) * (n_events + 1), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(E.sd_off, seed_offsets, sizeof(int32_t) * (n_events + 1), hipMemcpyHostToDevice));
    }
    const int32_t d[2] = {(int32_t)n_px, (int32_t)n_sd};
    HIPCHK(c, hipMemcpy((void *)(E.desc + D_NPX), d, sizeof(d), hipMemcpyHostToDevice));
    c->px_off.assign(px_offsets, px_offsets + n_events + 1);
    c->sd_off.assign(seed_offsets, seed_offsets + n_events + 1);
    // pixel constants, each rounded once from the double parameters
    PixConsts &P = c->pxk;
    const double wl = pp[LST_PX_WLINK] * c->params[LST_P_W];
    P.sig2p = (float)(pp[LST_PX_SIGRPHI] * pp[LST_PX_SIGRPHI]);
    P.sigz = (float)pp[LST_PX_SIGZ];
    P.wl2 = (float)(wl * wl);
    P.dr2 = (float)pp[LST_PX_DR2];
    P.x5p = (float)pp[LST_PX_X5P];
    P.x5z = (float)pp[LST_PX_X5Z];
    P.x3p = (float)pp[LST_PX_X3P];
    P.x3z = (float)pp[LST_PX_X3Z];
    // the window holds |dphi| <= asin(sqrt(wl2)) (same hemisphere); 1e-3 rad
    // covers the rounding of the directions' azimuths
    P.wphi = P.wl2 >= 1.0f ? 4.0f : (float)(std::asin(std::sqrt((double)P.wl2)) + 1e-3);
    // closeness holds sin^2(dphi) <= dr2 (same hemisphere)
    P.wdr = P.dr2 >= 1.0f ? 4.0f : (float)(std::asin(std::sqrt((double)P.dr2)) + 1e-3);
    c->px_loaded = true;
    c->counts_valid = false;
    return LST_OK;
}

// ---------------------------------------------------------------- stages
// Stage calls run in chain order.  Hit grouping (s = 1) may start a chain at
// any point after hits are loaded: it clears every object counter.  Each
// object stage and duplicate removal (s = 2..6) runs exactly once, right after
// its predecessor: running one again would append to the output ranges
// its first run reserved, and running it after a later stage would mix two
// chains' objects.
static int need_stage(lst_ctx *c, int s, const char *what)
{
    if (!c) return LST_E_INVALID;
    if (c->stage < s || (s >= 2 && c->stage != s))
        return fail(c, LST_E_STATE, "%s called out of order (chain at step %d)", what, c->stage);
    c->counts_valid = false;
    if (s <= 6) c->features_valid = false;
    if (s <= 5) c->t3_features_valid = false;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, LST_E_HIP, "hipSetDevice");
    return LST_OK;
}

static bool capped(const lst_ctx *c)
{
    return c->cap[OT_MD] > 0 || c->cap[OT_SEG] > 0 || c->cap[OT_T3] > 0 || c->cap[OT_T5] > 0;
}

// the capacity passes of one object type after its stage; the per-event drop
// counts are cleared before the first pass of a chain
static int enqueue_cap(lst_ctx *c, int type, hipStream_t s)
{
    if (!capped(c)) return LST_OK;
    if (type == OT_MD)
        HIPCHK(c, launch_zero(c->E, c->E.cap_nd,
                              (((size_t)c->E.cap_ev * OT_COUNT + 3) & ~(size_t)3) * sizeof(uint32_t), s));
    HIPCHK(c, launch_cap(c->E, type, c->cap[type], s));
    return LST_OK;
}

int lst_set_hit_storage(lst_ctx *c, int32_t fp16)
{
    if (!c) return LST_E_INVALID;
    if (fp16 != 0 && fp16 != 1) return fail(c, LST_E_INVALID, "hit storage %d (0 FP32, 1 FP16)", fp16);
    c->half16 = fp16;
    c->E.half16 = fp16;
    drop_graph(c);
    // hits grouped in the other storage are not readable: group them again
    if (c->stage > 1) c->stage = 1;
    c->counts_valid = false;
    return LST_OK;
}

int lst_set_capacities(lst_ctx *c, const int32_t *caps4)
{
    if (!c) return LST_E_INVALID;
    if (caps4)
        for (int t = 0; t < OT_COUNT; ++t)
            if (caps4[t] < 0) return fail(c, LST_E_INVALID, "capacity %d of kind %d", caps4[t], t);
    for (int t = 0; t < OT_COUNT; ++t) c->cap[t] = caps4 ? caps4[t] : 0;
    drop_graph(c);
    c->counts_valid = false;
    return LST_OK;
}

// scorer mode with no usable network: the batch runs the plain cut chain
// and its counts say so
static void note_fallback(lst_ctx *c)
{
    c->fallback = c->mode == LST_MODE_MLP && !c->mlp_dev[0] && !c->mlp_dev[1];
}

int lst_run_sort(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 1, "lst_run_sort");
    if (rc) return rc;
    note_fallback(c);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, launch_sort(c->E, c->M, c->tune.grid[ST_SORT], sort_per_event(c), s));
    c->stage = 2;
    return LST_OK;
}

int lst_run_md(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 2, "lst_run_md");
    if (rc) return rc;
    HIPCHK(c, launch_md(c->E, c->M, c->K, c->tune.grid[ST_MD], c->tune.lanes[ST_MD], (hipStream_t)stream));
    if ((rc = enqueue_cap(c, OT_MD, (hipStream_t)stream))) return rc;
    c->stage = 3;
    return LST_OK;
}

int lst_run_segments(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 3, "lst_run_segments");
    if (rc) return rc;
    HIPCHK(c, launch_seg(c->E, c->M, c->K, c->tune.grid[ST_SEG], c->tune.lanes[ST_SEG],
                         seg_share(c), (hipStream_t)stream));
    if ((rc = enqueue_cap(c, OT_SEG, (hipStream_t)stream))) return rc;
    c->stage = 4;
    return LST_OK;
}

int lst_run_triplets(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 4, "lst_run_triplets");
    if (rc) return rc;
    HIPCHK(c, launch_t3(c->E, c->M, c->K, c->tune.grid[ST_T3], c->tune.lanes[ST_T3], (hipStream_t)stream));
    if ((rc = enqueue_cap(c, OT_T3, (hipStream_t)stream))) return rc;
    c->stage = 5;
    return LST_OK;
}

int lst_run_quintuplets(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 5, "lst_run_quintuplets");
    if (rc) return rc;
    HIPCHK(c, launch_t5(c->E, c->M, c->K, c->tune.grid[ST_T5], c->tune.lanes[ST_T5], (hipStream_t)stream));
    if ((rc = enqueue_cap(c, OT_T5, (hipStream_t)stream))) return rc;
    c->stage = 6;
    return LST_OK;
}

int lst_run_dedup(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 6, "lst_run_dedup");
    if (rc) return rc;
    HIPCHK(c, launch_dedup(c->E, c->M, c->tune.grid[ST_DEDUP], (hipStream_t)stream));
    c->stage = 7;
    return LST_OK;
}

int lst_run_chain_persistent(lst_ctx *c, void *stream);

int lst_run_pixel(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 7, "lst_run_pixel");
    if (rc) return rc;
    if (!c->px_loaded) return fail(c, LST_E_STATE, "no pixel seeds loaded for this batch");
    HIPCHK(c, launch_pixel(c->E, c->K, c->pxk, (hipStream_t)stream));
    c->stage = 8;
    return LST_OK;
}

// ---------------------------------------------------------------- learned scorer
static int score_grid(const lst_ctx *c, int slot);
static int enqueue_score(lst_ctx *c, int slot, hipStream_t s);

static int mlp_slot(int32_t kind) { return kind == LST_T3 ? 0 : kind == LST_T5 ? 1 : -1; }

int lst_set_mode(lst_ctx *c, int32_t mode)
{
    if (!c) return LST_E_INVALID;
    if (mode != LST_MODE_CUTS && mode != LST_MODE_MLP) return fail(c, LST_E_INVALID, "mode %d", mode);
    if (mode != c->mode) drop_graph(c);
    c->mode = mode;
    return LST_OK;
}

int lst_mlp_load(lst_ctx *c, int32_t kind, const float *params, int32_t n_params, const float *mean,
                 const float *istd, float threshold)
{
    if (!c) return LST_E_INVALID;
    const int sl = mlp_slot(kind);
    if (sl < 0) return fail(c, LST_E_INVALID, "scorer kind %d (LST_T3 or LST_T5)", kind);
    HIPCHK(c, hipSetDevice(c->device));
    // rejected weights also unload the kind's earlier network: that stage
    // then runs its plain cuts
    auto reject = [&](const char *what, int i) {
        char msg[96];
        std::snprintf(msg, sizeof msg, what, i);
        if (c->mlp_dev[sl]) {
            drop_graph(c);
            (void)hipDeviceSynchronize();
            (void)hipFree(c->mlp_dev[sl]);
            c->mlp_dev[sl] = nullptr;
        }
        return fail(c, LST_E_INVALID, "%s", msg);
    };
    if (!params || !mean || !istd || n_params != MLP_NPARAM)
        return reject("scorer weights: %d parameters expected", MLP_NPARAM);
    for (int i = 0; i < MLP_NPARAM; ++i)
        if (!std::isfinite(params[i])) return reject("scorer parameter %d not finite", i);
    for (int i = 0; i < MLP_NIN; ++i)
        if (!std::isfinite(mean[i]) || !std::isfinite(istd[i]))
            return reject("standardisation of feature %d not finite", i);
    if (!std::isfinite(threshold)) return reject("threshold not finite (kind slot %d)", sl);
    const size_t n = MLP_NPARAM + 2 * MLP_NIN;
    const bool fresh = !c->mlp_dev[sl];
    if (fresh) HIPCHK(c, hipMalloc((void **)&c->mlp_dev[sl], sizeof(float) * n));
    std::vector<float> h(n);
    std::memcpy(h.data(), params, sizeof(float) * MLP_NPARAM);
    std::memcpy(h.data() + MLP_NPARAM, mean, sizeof(float) * MLP_NIN);
    std::memcpy(h.data() + MLP_NPARAM + MLP_NIN, istd, sizeof(float) * MLP_NIN);
    // synchronous: a replayed graph reads these weights by address
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(c->mlp_dev[sl], h.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    if (fresh || threshold != c->mlp_threshold[sl]) drop_graph(c);
    c->mlp_threshold[sl] = threshold;
    return LST_OK;
}

int lst_run_t3_score(lst_ctx *c, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (!c->mlp_dev[0]) return fail(c, LST_E_STATE, "triplet scorer weights not loaded");
    if (c->stage != 5)
        return fail(c, LST_E_STATE, "lst_run_t3_score runs after triplets, before quintuplets");
    int rc = need_stage(c, 5, "lst_run_t3_score");
    if (rc) return rc;
    return enqueue_score(c, 0, (hipStream_t)stream);
}

int lst_run_t5_score(lst_ctx *c, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (!c->mlp_dev[1]) return fail(c, LST_E_STATE, "quintuplet scorer weights not loaded");
    if (c->stage != 6)
        return fail(c, LST_E_STATE, "lst_run_t5_score runs after quintuplets, before dedup");
    int rc = need_stage(c, 6, "lst_run_t5_score");
    if (rc) return rc;
    return enqueue_score(c, 1, (hipStream_t)stream);
}

size_t lst_mlp_workspace_bytes(int64_t n) { return n < 0 ? 0 : mlp_workspace_bytes(n); }

static int mlp_args(lst_ctx *c, int64_t n, std::initializer_list<const void *> ptrs)
{
    if (!c) return LST_E_INVALID;
    if (n < 0 || n > ((int64_t)1 << 31)) return fail(c, LST_E_INVALID, "rows %lld", (long long)n);
    if (n > 0)   // empty batches may come with null pointers
        for (const void *p : ptrs)
            if (!p) return fail(c, LST_E_INVALID, "null device pointer");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, LST_E_HIP, "hipSetDevice");
    return LST_OK;
}

int lst_mlp_prepare(lst_ctx *c, const float *feat, const float *mean, const float *istd, int64_t n,
                    uint16_t *x, void *stream)
{
    int rc = mlp_args(c, n, {feat, mean, istd, x});
    if (rc || n == 0) return rc;
    HIPCHK(c, mlp_prepare(feat, mean, istd, n, x, (hipStream_t)stream));
    return LST_OK;
}

int lst_mlp_forward(lst_ctx *c, const float *params, const uint16_t *x, int64_t n, float *logits,
                    uint16_t *h1, float *h2, void *stream)
{
    int rc = mlp_args(c, n, {params, x, logits});
    if (rc || n == 0) return rc;
    if (!h1 != !h2) return fail(c, LST_E_INVALID, "h1 and h2 are saved together");
    HIPCHK(c, mlp_forward(params, x, n, logits, h1, h2, (hipStream_t)stream));
    return LST_OK;
}

int lst_mlp_backward(lst_ctx *c, const float *params, const uint16_t *x, const uint8_t *y, int64_t n,
                     const float *logits, const uint16_t *h1, const float *h2, void *work,
                     size_t work_bytes, float *grad, float *loss, void *stream)
{
    int rc = mlp_args(c, n, {params, x, y, logits, h1, h2, work, grad, loss});
    if (rc) return rc;
    if (n == 0) return fail(c, LST_E_INVALID, "empty batch");
    if (work_bytes < mlp_workspace_bytes(n))
        return fail(c, LST_E_CAPACITY, "workspace %zu bytes, %zu needed", work_bytes,
                    mlp_workspace_bytes(n));
    HIPCHK(c, mlp_backward(params, x, y, n, logits, h1, h2, (float *)work, grad, loss,
                           (hipStream_t)stream));
    return LST_OK;
}

int lst_mlp_backward_noalloc(lst_ctx *c, const float *params, const uint16_t *x, const uint8_t *y,
                             int64_t n, const float *logits, const uint16_t *h1, const float *h2,
                             float *grad, float *loss, void *stream)
{
    int rc = mlp_args(c, n, {params, x, y, logits, h1, h2, grad, loss});
    if (rc) return rc;
    if (n == 0) return fail(c, LST_E_INVALID, "empty batch");
    if (n > MLP_FIXED_MAX_ROWS)
        return fail(c, LST_E_CAPACITY, "%lld rows: the fixed workspace holds at most %lld",
                    (long long)n, (long long)MLP_FIXED_MAX_ROWS);
    // every workspace word the kernels read is written by them first in the
    // same call: nothing to clear
    HIPCHK(c, mlp_backward(params, x, y, n, logits, h1, h2, (float *)c->fixed_work, grad, loss,
                           (hipStream_t)stream));
    return LST_OK;
}

int lst_mlp_adam(lst_ctx *c, float *params, const float *grad, float *m, float *v, int32_t step,
                 float lr, float beta1, float beta2, float eps, void *stream)
{
    int rc = mlp_args(c, MLP_NPARAM, {params, grad, m, v});
    if (rc) return rc;
    if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(c, LST_E_INVALID, "Adam hyper-parameters");
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    HIPCHK(c, mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream));
    return LST_OK;
}

int lst_mlp_train_steps(lst_ctx *c, float *params, const uint16_t *x, const uint8_t *y,
                        int64_t n_rows, int64_t batch, const int32_t *order, int32_t n_steps,
                        int32_t first_step, float *logits, uint16_t *h1, float *h2, void *work,
                        size_t work_bytes, float *grad, float *m, float *v, float *losses,
                        float lr, float beta1, float beta2, float eps, void *stream)
{
    (void)logits;   // the forward runs inside the gradient kernel
    (void)h1;
    (void)h2;
    int rc = mlp_args(c, batch, {params, x, y, work, grad, m, v, losses});
    if (rc) return rc;
    if (batch < 1 || n_rows < batch || n_steps < 0 || first_step < 0 || (n_steps > 0 && !order))
        return fail(c, LST_E_INVALID, "rows %lld, batch %lld, steps %d from %d", (long long)n_rows,
                    (long long)batch, n_steps, first_step);
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(c, LST_E_INVALID, "Adam hyper-parameters");
    if (work_bytes < mlp_workspace_bytes(batch))
        return fail(c, LST_E_CAPACITY, "workspace %zu bytes, %zu needed", work_bytes,
                    mlp_workspace_bytes(batch));
    const int64_t n_batches = n_rows / batch;
    for (int32_t i = 0; i < n_steps; ++i)
        if (order[i] < 0 || order[i] >= n_batches)
            return fail(c, LST_E_INVALID, "order[%d] = %d outside 0..%lld", i, order[i],
                        (long long)n_batches - 1);
    const hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < n_steps; ++i) {
        const int64_t r0 = (int64_t)order[i] * batch;
        const uint16_t *xb = x + r0 * 64;
        const uint8_t *yb = y + r0;
        // bias corrections exactly as lst_mlp_adam computes them
        const int32_t step = first_step + 1 + i;
        const float c1 = (float)(1.0 - std::pow((double)beta1, step));
        const float c2 = (float)(1.0 - std::pow((double)beta2, step));
        // forward, backward and Adam in two launches with the same arithmetic
        HIPCHK(c, mlp_train_step(params, xb, yb, batch, (float *)work, grad, losses + order[i], m,
                                 v, lr, beta1, beta2, eps, c1, c2, s));
    }
    return LST_OK;
}

int lst_run_chain(lst_ctx *c, void *stream)
{
    int rc;
    if (c && c->tune.persistent && !capped(c)) return lst_run_chain_persistent(c, stream);
    if ((rc = lst_run_sort(c, stream))) return rc;
    if ((rc = lst_run_md(c, stream))) return rc;
    if ((rc = lst_run_segments(c, stream))) return rc;
    if ((rc = lst_run_triplets(c, stream))) return rc;
    const bool mlp = c->mode == LST_MODE_MLP;
    if (mlp && c->mlp_dev[0] && (rc = lst_run_t3_score(c, stream))) return rc;
    if ((rc = lst_run_quintuplets(c, stream))) return rc;
    if (mlp && c->mlp_dev[1] && (rc = lst_run_t5_score(c, stream))) return rc;
    return lst_run_dedup(c, stream);
}

// The whole chain as one hipGraph: captured once per arena (kernel grids and
// arguments depend on the arena only; batch sizes are read on the device)
// and replayed for every batch.  Only kernel nodes: no memset nodes.
static int score_grid(const lst_ctx *c, int slot)
{
    // one block scores 256 objects per pass; grid-stride beyond that
    const int64_t cap = slot == 0 ? c->caps.t3 : c->caps.t5;
    const int64_t need = (cap + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, 2 * std::max(c->n_cu, 1)));
}

static int enqueue_score(lst_ctx *c, int slot, hipStream_t s)
{
    const float *P = c->mlp_dev[slot];
    HIPCHK(c, mlp_score(c->E, c->K, slot == 0 ? OT_T3 : OT_T5, P, P + MLP_NPARAM,
                        P + MLP_NPARAM + MLP_NIN, c->mlp_threshold[slot], score_grid(c, slot), s));
    return LST_OK;
}

// the stages after a persistent launch that stopped early for scoring
static int enqueue_after_persistent(lst_ctx *c, int stop, hipStream_t s)
{
    const Tuning &t = c->tune;
    int rc;
    if (stop == PERS_TO_T3) {
        if ((rc = enqueue_score(c, 0, s))) return rc;
        HIPCHK(c, launch_t5(c->E, c->M, c->K, t.grid[ST_T5], t.lanes[ST_T5], s));
    }
    if (c->mlp_dev[1] && (rc = enqueue_score(c, 1, s))) return rc;
    HIPCHK(c, launch_dedup(c->E, c->M, t.grid[ST_DEDUP], s));
    return LST_OK;
}

static int persistent_stop(const lst_ctx *c)
{
    if (c->mode != LST_MODE_MLP) return PERS_FULL;
    return c->mlp_dev[0] ? PERS_TO_T3 : c->mlp_dev[1] ? PERS_TO_T5 : PERS_FULL;
}

static int enqueue_chain(lst_ctx *c, hipStream_t s)
{
    const Tuning &t = c->tune;
    const bool mlp = c->mode == LST_MODE_MLP;
    int rc;
    if (t.persistent && !capped(c)) {
        const int stop = persistent_stop(c);
        HIPCHK(c, launch_chain_persistent(c->E, c->M, c->K, c->zero_base, c->zero_bytes,
                                          t.blocks_per_cu * c->n_cu, t.lanes[ST_SEG], stop, s));
        return stop == PERS_FULL ? LST_OK : enqueue_after_persistent(c, stop, s);
    }
    HIPCHK(c, launch_sort(c->E, c->M, t.grid[ST_SORT], sort_per_event(c), s));
    HIPCHK(c, launch_md(c->E, c->M, c->K, t.grid[ST_MD], t.lanes[ST_MD], s));
    if ((rc = enqueue_cap(c, OT_MD, s))) return rc;
    HIPCHK(c, launch_seg(c->E, c->M, c->K, t.grid[ST_SEG], t.lanes[ST_SEG], seg_share(c), s));
    if ((rc = enqueue_cap(c, OT_SEG, s))) return rc;
    HIPCHK(c, launch_t3(c->E, c->M, c->K, t.grid[ST_T3], t.lanes[ST_T3], s));
    if ((rc = enqueue_cap(c, OT_T3, s))) return rc;
    if (mlp && c->mlp_dev[0] && (rc = enqueue_score(c, 0, s))) return rc;
    HIPCHK(c, launch_t5(c->E, c->M, c->K, t.grid[ST_T5], t.lanes[ST_T5], s));
    if ((rc = enqueue_cap(c, OT_T5, s))) return rc;
    if (mlp && c->mlp_dev[1] && (rc = enqueue_score(c, 1, s))) return rc;
    HIPCHK(c, launch_dedup(c->E, c->M, t.grid[ST_DEDUP], s));
    return LST_OK;
}

int lst_run_chain_persistent(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 1, "lst_run_chain_persistent");
    if (rc) return rc;
    note_fallback(c);
    if (capped(c))
        return fail(c, LST_E_STATE, "per-module capacities run with the per-stage chain only");
    const int bpc =
        std::max(1, std::min(c->tune.blocks_per_cu, persistent_blocks_per_cu(c->tune.lanes[ST_SEG])));
    hipStream_t s = (hipStream_t)stream;
    const int stop = persistent_stop(c);
    HIPCHK(c, launch_chain_persistent(c->E, c->M, c->K, c->zero_base, c->zero_bytes,
                                      bpc * c->n_cu, c->tune.lanes[ST_SEG], stop, s));
    if (stop != PERS_FULL && (rc = enqueue_after_persistent(c, stop, s))) return rc;
    c->stage = 7;
    return LST_OK;
}

// feature passes read finished stages; they invalidate nothing else
int lst_run_t3_features(lst_ctx *c, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (c->stage < 5) return fail(c, LST_E_STATE, "lst_run_t3_features called out of order");
    HIPCHK(c, hipSetDevice(c->device));
    if (!c->E.t3_feat) return fail(c, LST_E_STATE, "arena attached without features");
    HIPCHK(c, launch_t3_features(c->E, c->K, c->tune.grid[ST_DEDUP], (hipStream_t)stream));
    c->t3_features_valid = true;
    return LST_OK;
}

int lst_run_t5_features(lst_ctx *c, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (c->stage < 6) return fail(c, LST_E_STATE, "lst_run_t5_features called out of order");
    HIPCHK(c, hipSetDevice(c->device));
    if (!c->E.t5_feat) return fail(c, LST_E_STATE, "arena attached without features");
    HIPCHK(c, launch_t5_features(c->E, c->K, c->tune.grid[ST_DEDUP], (hipStream_t)stream));
    c->features_valid = true;
    return LST_OK;
}

static bool lanes_ok(int v) { return v == 8 || v == 16 || v == 32 || v == 64; }

int lst_set_tuning(lst_ctx *c, const int32_t *grid6, const int32_t *lanes6, int32_t persistent,
                   int32_t blocks_per_cu)
{
    if (!c || !grid6) return LST_E_INVALID;
    if (!c->arena) return fail(c, LST_E_STATE, "no arena attached");
    for (int i = 0; i < ST_COUNT; ++i)
        if (grid6[i] < 1 || grid6[i] > 65535) return fail(c, LST_E_INVALID, "grid[%d] = %d", i, grid6[i]);
    if (lanes6)
        for (int i = 0; i < ST_COUNT; ++i)
            if (!lanes_ok(lanes6[i])) return fail(c, LST_E_INVALID, "lanes[%d] = %d", i, lanes6[i]);
    const int occ = persistent_blocks_per_cu(lanes6 ? lanes6[ST_SEG] : c->tune.lanes[ST_SEG]);
    if (blocks_per_cu < 1 || blocks_per_cu > occ)
        return fail(c, LST_E_INVALID, "blocks_per_cu %d outside 1..%d (co-residency)", blocks_per_cu, occ);
    for (int i = 0; i < ST_COUNT; ++i) {
        c->tune.grid[i] = grid6[i];
        if (lanes6) c->tune.lanes[i] = lanes6[i];
    }
    c->tune.persistent = persistent ? 1 : 0;
    c->tune.blocks_per_cu = blocks_per_cu;
    drop_graph(c);
    return LST_OK;
}

int lst_get_tuning(const lst_ctx *c, int32_t *out15)
{
    if (!c || !out15) return LST_E_INVALID;
    for (int i = 0; i < ST_COUNT; ++i) {
        out15[i] = c->tune.grid[i];
        out15[ST_COUNT + i] = c->tune.lanes[i];
    }
    out15[12] = c->tune.persistent;
    out15[13] = c->tune.blocks_per_cu;
    out15[14] = c->n_cu;
    return LST_OK;
}

int lst_run_chain_graph(lst_ctx *c, void *stream)
{
    int rc = need_stage(c, 1, "lst_run_chain_graph");
    if (rc) return rc;
    note_fallback(c);
    if (!c->graph) {
        if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        rc = enqueue_chain(c, c->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(c, LST_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph = nullptr;
            return fail(c, LST_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    HIPCHK(c, hipGraphLaunch(c->graph, (hipStream_t)stream));
    c->stage = 7;
    return LST_OK;
}

// ---------------------------------------------------------------- results
static int sync_stream(lst_ctx *c, void *stream)
{
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    HIPCHK(c, hipGetLastError());
    return LST_OK;
}

int lst_stream_copy(void *dst, const void *src, size_t n_bytes, void *stream)
{
    if (!dst || !src || (n_bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return LST_E_INVALID;
    if (launch_copy(dst, src, n_bytes, (hipStream_t)stream) != hipSuccess) return LST_E_HIP;
    return LST_OK;
}

}  // extern "C"

// Shard counters of every object type, read back from the device.
struct ShardCounts {
    uint32_t gc[GC_COUNT];
    uint32_t rc[OT_COUNT];
    uint32_t n(int t, int s) const { return std::min(gc[gc_shard(t, s)], rc[t]); }
    size_t span(int t) const { return (size_t)rc[t] * NSH; }
    // capacity that would have let every shard fit
    int64_t required(int t) const
    {
        uint32_t m = 0;
        for (int s = 0; s < NSH; ++s) m = std::max(m, gc[gc_shard(t, s)]);
        return (int64_t)m * NSH;
    }
    int64_t stored(int t) const
    {
        int64_t k = 0;
        for (int s = 0; s < NSH; ++s) k += n(t, s);
        return k;
    }
};

static int read_shards(lst_ctx *c, ShardCounts &S)
{
    HIPCHK(c, hipMemcpy(S.gc, c->E.gc, sizeof(S.gc), hipMemcpyDeviceToHost));
    std::memcpy(S.rc, c->E.rc, sizeof(S.rc));
    return LST_OK;
}

// Error bits 1 (a persistent-chain grid barrier timed out) and 2 (the
// grouping scan timed out) make the outputs unusable and can leave bin
// counts non-zero, while the grouping of the next chain relies on them being
// zero: the bins are cleared here.  The error word itself stays set until the
// next chain clears it, so every getter keeps refusing until then.
static int check_fault(lst_ctx *c, uint32_t err)
{
    if (!(err & 6u)) return LST_OK;
    char *b = (char *)c->E.bcnt;
    const size_t n = (size_t)((char *)c->zero_base + c->zero_bytes - b);
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, launch_zero(c->E, b, n, nullptr));
    HIPCHK(c, hipDeviceSynchronize());
    return fail(c, LST_E_FAULT, "a kernel-side wait timed out (error flags %u): the outputs are unusable",
                err);
}

// Per-event statistics, reduced on the host from the device arrays (the
// reporting path; the stage kernels carry no statistics atomics).
static int compute_counts(lst_ctx *c)
{
    const EvDev &E = c->E;
    const int n_ev = c->n_events, nm = c->n_mod;
    ShardCounts S;
    int rc = read_shards(c, S);
    if (rc) return rc;
    c->counts.assign(n_ev, lst_counts{});
    for (int e = 0; e < n_ev; ++e) {
        c->counts[e].n_hits = c->hit_off[e + 1] - c->hit_off[e];
        c->counts[e].overflow_mask = (int32_t)S.gc[GC_OVERFLOW];
        c->counts[e].error_flags = (int32_t)S.gc[GC_ERROR];
        c->counts[e].mlp_fallback = c->fallback ? 1 : 0;
    }
    if (capped(c) && c->stage >= 3) {
        std::vector<uint32_t> nd;
        if ((rc = d2h(c, nd, E.cap_nd, (size_t)n_ev * OT_COUNT))) return rc;
        // a kind's counts are only meaningful once its stage (and pass) ran
        for (int e = 0; e < n_ev; ++e)
            for (int t = 0; t < OT_COUNT; ++t)
                c->counts[e].dropped[t] = c->stage >= 3 + t ? nd[(size_t)e * OT_COUNT + t] : 0;
    }
    if (S.gc[GC_OVERFLOW]) {
        // arrays are incomplete: report the batch-wide requirement instead
        for (auto &k : c->counts) {
            k.n_md = S.required(OT_MD);
            k.n_seg = S.required(OT_SEG);
            k.n_t3 = S.required(OT_T3);
            k.n_t5 = S.required(OT_T5);
        }
        c->counts_valid = true;
        return LST_OK;
    }
    const size_t slots = (size_t)n_ev * nm;
    std::vector<uint32_t> boff;
    std::vector<int32_t> mds, mdc, mslot, ss, sc, so, ts, tc, tcc, t50;
    std::vector<uint8_t> keep;
    const size_t nmd = S.span(OT_MD), nseg = S.span(OT_SEG), nt3 = S.span(OT_T3), nt5 = S.span(OT_T5);
    if ((rc = d2h(c, boff, E.boff, 2 * slots + 1)) || (rc = d2h(c, mds, E.md_start, slots)) ||
        (rc = d2h(c, mdc, E.md_cnt, slots)))
        return rc;
    if (c->stage >= 3 && (rc = d2h(c, mslot, E.md_slot, nmd))) return rc;
    if (c->stage >= 4 && ((rc = d2h(c, ss, E.seg_start, nmd)) || (rc = d2h(c, sc, E.seg_cnt, nmd)) ||
                          (rc = d2h(c, so, E.seg_out, nseg))))
        return rc;
    if (c->stage >= 5 && ((rc = d2h(c, ts, E.t3_start, nmd)) || (rc = d2h(c, tc, E.t3_cnt, nmd)) ||
                          (rc = d2h(c, tcc, E.t3_c, nt3))))
        return rc;
    if (c->stage >= 6 && (rc = d2h(c, t50, E.t5_md0, nt5))) return rc;
    if (c->stage >= 7 && (rc = d2h(c, keep, E.t5_keep, nt5))) return rc;
    for (int e = 0; e < n_ev; ++e) {
        lst_counts &k = c->counts[e];
        for (int m = 0; m < nm; ++m) {
            const size_t sl = (size_t)e * nm + m;
            const int64_t nlo = boff[2 * sl + 1] - boff[2 * sl];
            const int64_t nup = boff[2 * sl + 2] - boff[2 * sl + 1];
            k.cand_md += nlo * nup;
            if (c->stage < 3 || mdc[sl] == 0) continue;
            k.n_md += mdc[sl];
            int64_t outer = 0;
            for (int32_t q = c->map_ptr[m]; q < c->map_ptr[m + 1]; ++q)
                outer += mdc[(size_t)e * nm + c->map_col[q]];
            k.cand_seg += (int64_t)mdc[sl] * outer;
            if (c->stage < 4) continue;
            for (int32_t a = mds[sl]; a < mds[sl] + mdc[sl]; ++a) {
                k.n_seg += sc[a];
                for (int32_t s1 = ss[a]; s1 < ss[a] + sc[a]; ++s1) k.cand_t3 += sc[so[s1]];
                if (c->stage < 5) continue;
                k.n_t3 += tc[a];
                for (int32_t t1 = ts[a]; t1 < ts[a] + tc[a]; ++t1) k.cand_t5 += tc[tcc[t1]];
            }
        }
    }
    std::vector<uint8_t> clean;
    if (c->stage >= 8 && (rc = d2h(c, clean, E.t5_clean, nt5))) return rc;
    if (c->stage >= 6) {
        for (int s = 0; s < NSH; ++s)
            for (uint32_t q = 0; q < S.n(OT_T5, s); ++q) {
                const size_t t = (size_t)s * S.rc[OT_T5] + q;
                const int e = mslot[t50[t]] / nm;
                c->counts[e].n_t5++;
                if (c->stage >= 7) c->counts[e].n_t5_kept += keep[t];
                if (c->stage >= 8) c->counts[e].n_tc += clean[t];
            }
    }
    if (c->stage >= 8) {
        const uint32_t n5 = std::min<uint32_t>(S.gc[GC_PX5], (uint32_t)E.cap_pxc);
        const uint32_t n3 = std::min<uint32_t>(S.gc[GC_PX3], (uint32_t)E.cap_pxc);
        const int64_t n_sd = c->sd_off[n_ev];
        std::vector<int32_t> s5, s3, sev;
        std::vector<uint8_t> k5, k3, sk;
        if ((rc = d2h(c, s5, E.c5_seed, n5)) || (rc = d2h(c, k5, E.c5_keep, n5)) ||
            (rc = d2h(c, s3, E.c3_seed, n3)) || (rc = d2h(c, k3, E.c3_keep, n3)) ||
            (rc = d2h(c, sev, E.sd_ev, n_sd)) || (rc = d2h(c, sk, E.sd_keep, n_sd)))
            return rc;
        for (int e = 0; e < n_ev; ++e) c->counts[e].n_pls = c->sd_off[e + 1] - c->sd_off[e];
        for (uint32_t i = 0; i < n5; ++i) {
            lst_counts &k = c->counts[sev[s5[i]]];
            k.cand_pt5++;
            k.n_pt5 += k5[i];
            k.n_tc += k5[i];
        }
        for (uint32_t i = 0; i < n3; ++i) {
            lst_counts &k = c->counts[sev[s3[i]]];
            k.cand_pt3++;
            k.n_pt3 += k3[i];
            k.n_tc += k3[i];
        }
        for (int64_t q = 0; q < n_sd; ++q) c->counts[sev[q]].n_tc += sk[q];
    }
    c->counts_valid = true;
    return LST_OK;
}

extern "C" {

int lst_get_counts(lst_ctx *c, int32_t event, lst_counts *out, void *stream)
{
    if (!c || !out) return LST_E_INVALID;
    if (c->stage < 2) return fail(c, LST_E_STATE, "no chain has run");
    if (event < 0 || event >= c->n_events) return fail(c, LST_E_INVALID, "event %d", event);
    int rc = sync_stream(c, stream);
    if (rc) return rc;
    if (!c->counts_valid && (rc = compute_counts(c))) return rc;
    *out = c->counts[event];
    if ((rc = check_fault(c, (uint32_t)out->error_flags))) return rc;
    if (out->overflow_mask)
        return fail(c, LST_E_CAPACITY,
                    "capacity overflow (mask %d): MD %lld SEG %lld T3 %lld T5 %lld needed",
                    out->overflow_mask, (long long)out->n_md, (long long)out->n_seg,
                    (long long)out->n_t3, (long long)out->n_t5);
    return LST_OK;
}

int lst_raise_error_flags(lst_ctx *c, int32_t bits, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (bits & ~6) return fail(c, LST_E_INVALID, "only error bits 1 and 2 may be raised (%d)", bits);
    if (c->stage < 2) return fail(c, LST_E_STATE, "no chain has run");
    int rc = sync_stream(c, stream);
    if (rc) return rc;
    uint32_t w = 0;
    HIPCHK(c, hipMemcpy(&w, &c->E.gc[GC_ERROR], sizeof(w), hipMemcpyDeviceToHost));
    w |= (uint32_t)bits;
    HIPCHK(c, hipMemcpy(&c->E.gc[GC_ERROR], &w, sizeof(w), hipMemcpyHostToDevice));
    c->counts_valid = false;
    return LST_OK;
}

int lst_get_objects(lst_ctx *c, int32_t event, int32_t kind, int32_t *out, int64_t cap,
                    int64_t *n_tuples, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (kind < LST_MD || kind > LST_T5_KEPT) return fail(c, LST_E_INVALID, "kind %d", kind);
    if (event < 0 || event >= c->n_events) return fail(c, LST_E_INVALID, "event %d", event);
    const int need = kind == LST_MD ? 3 : kind == LST_SEG ? 4 : kind == LST_T3 ? 5 : kind == LST_T5 ? 6 : 7;
    if (c->stage < need) return fail(c, LST_E_STATE, "stage for kind %d has not run", kind);
    int rc = sync_stream(c, stream);
    if (rc) return rc;
    const EvDev &E = c->E;
    ShardCounts S;
    if ((rc = read_shards(c, S)) || (rc = check_fault(c, S.gc[GC_ERROR]))) return rc;
    if (S.gc[GC_OVERFLOW])
        return fail(c, LST_E_CAPACITY, "capacity overflow (mask %u)", S.gc[GC_OVERFLOW]);
    const size_t n_sorted = S.gc[GC_N_SORTED];
    const size_t nmd = S.span(OT_MD);
    std::vector<int32_t> sorig, hlo, hup, slot;
    if ((rc = sorted_orig(c, sorig, n_sorted)) || (rc = d2h(c, hlo, E.md_hlo, nmd)) ||
        (rc = d2h(c, hup, E.md_hup, nmd)) || (rc = d2h(c, slot, E.md_slot, nmd)))
        return rc;
    const int lo_slot = event * c->n_mod, hi_slot = (event + 1) * c->n_mod;
    auto in_ev = [&](int32_t md) { return slot[md] >= lo_slot && slot[md] < hi_slot; };
    auto put = [&](std::vector<int32_t> &tup, int32_t md) {
        tup.push_back(sorig[hlo[md]]);
        tup.push_back(sorig[hup[md]]);
    };
    std::vector<int32_t> tup;
    int width = 2;
    const int type = kind == LST_MD ? OT_MD : kind == LST_SEG ? OT_SEG : kind == LST_T3 ? OT_T3 : OT_T5;
    const size_t sp = S.span(type);
    std::vector<int32_t> a, b, d, e4, f5;
    std::vector<uint8_t> keep;
    if (kind == LST_SEG) {
        width = 4;
        if ((rc = d2h(c, a, E.seg_in, sp)) || (rc = d2h(c, b, E.seg_out, sp))) return rc;
    } else if (kind == LST_T3) {
        width = 6;
        if ((rc = d2h(c, a, E.t3_a, sp)) || (rc = d2h(c, b, E.t3_b, sp)) || (rc = d2h(c, d, E.t3_c, sp)))
            return rc;
    } else if (kind >= LST_T5) {
        width = 10;
        if ((rc = d2h(c, a, E.t5_md0, sp)) || (rc = d2h(c, b, E.t5_md1, sp)) ||
            (rc = d2h(c, d, E.t5_md2, sp)) || (rc = d2h(c, e4, E.t5_md3, sp)) ||
            (rc = d2h(c, f5, E.t5_md4, sp)) || (rc = d2h(c, keep, E.t5_keep, sp)))
            return rc;
    }
    for (int s = 0; s < NSH; ++s) {
        for (uint32_t q = 0; q < S.n(type, s); ++q) {
            const size_t i = (size_t)s * S.rc[type] + q;
            if (kind == LST_MD) {
                if (in_ev((int32_t)i)) put(tup, (int32_t)i);
            } else if (kind == LST_SEG) {
                if (in_ev(a[i])) { put(tup, a[i]); put(tup, b[i]); }
            } else if (kind == LST_T3) {
                if (in_ev(a[i])) { put(tup, a[i]); put(tup, b[i]); put(tup, d[i]); }
            } else {
                if (!in_ev(a[i]) || (kind == LST_T5_KEPT && !keep[i])) continue;
                put(tup, a[i]); put(tup, b[i]); put(tup, d[i]); put(tup, e4[i]); put(tup, f5[i]);
            }
        }
    }
    const int64_t nt = (int64_t)tup.size() / width;
    if (n_tuples) *n_tuples = nt;
    if (nt > cap)
        return fail(c, LST_E_CAPACITY, "%lld tuples, capacity %lld", (long long)nt, (long long)cap);
    if (out && nt) std::memcpy(out, tup.data(), sizeof(int32_t) * tup.size());
    return LST_OK;
}


}  // extern "C"

// copy a per-object device array (width values per object) of `event` in
// lst_get_objects order, for triplets (OT_T3) or quintuplets (OT_T5)
template <class T>
static int obj_field(lst_ctx *c, int type, int32_t event, const T *src, int width, T *out,
                     int64_t cap, int64_t *n_out, void *stream, const char *what)
{
    if (!c) return LST_E_INVALID;
    if (event < 0 || event >= c->n_events) return fail(c, LST_E_INVALID, "event %d", event);
    if (c->stage < (type == OT_T3 ? 5 : 6)) return fail(c, LST_E_STATE, "objects have not been built");
    int rc = sync_stream(c, stream);
    if (rc) return rc;
    const EvDev &E = c->E;
    ShardCounts S;
    if ((rc = read_shards(c, S)) || (rc = check_fault(c, S.gc[GC_ERROR]))) return rc;
    if (S.gc[GC_OVERFLOW])
        return fail(c, LST_E_CAPACITY, "capacity overflow (mask %u)", S.gc[GC_OVERFLOW]);
    std::vector<int32_t> m0, slot;
    std::vector<T> val;
    if ((rc = d2h(c, m0, type == OT_T3 ? E.t3_a : E.t5_md0, S.span(type))) ||
        (rc = d2h(c, val, src, S.span(type) * width)) || (rc = d2h(c, slot, E.md_slot, S.span(OT_MD))))
        return rc;
    const int lo_slot = event * c->n_mod, hi_slot = (event + 1) * c->n_mod;
    int64_t k = 0;
    for (int sh = 0; sh < NSH; ++sh)
        for (uint32_t q = 0; q < S.n(type, sh); ++q) {
            const size_t i = (size_t)sh * S.rc[type] + q;
            if (slot[m0[i]] < lo_slot || slot[m0[i]] >= hi_slot) continue;
            if (out && k < cap) std::memcpy(&out[width * k], &val[width * i], width * sizeof(T));
            ++k;
        }
    if (n_out) *n_out = k;
    if (k > cap)
        return fail(c, LST_E_CAPACITY, "%lld %s, capacity %lld", (long long)k, what, (long long)cap);
    return LST_OK;
}

extern "C" {

int lst_get_t5_scores(lst_ctx *c, int32_t event, float *out, int64_t cap, int64_t *n_out,
                      void *stream)
{
    return obj_field(c, OT_T5, event, c ? c->E.t5_score : nullptr, 1, out, cap, n_out, stream,
                     "scores");
}

int lst_get_t5_logits(lst_ctx *c, int32_t event, float *logits, uint8_t *veto, int64_t cap,
                      int64_t *n_out, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (c->stage < 7 && c->stage != 6) return fail(c, LST_E_STATE, "quintuplets have not run");
    int rc = obj_field(c, OT_T5, event, c->E.t5_logit, 1, logits, cap, n_out, stream, "logits");
    if (rc) return rc;
    return obj_field(c, OT_T5, event, c->E.t5_veto, 1, veto, cap, n_out, stream, "vetoes");
}

int lst_get_t3_logits(lst_ctx *c, int32_t event, float *logits, uint8_t *veto, int64_t cap,
                      int64_t *n_out, void *stream)
{
    if (!c) return LST_E_INVALID;
    int rc = obj_field(c, OT_T3, event, c->E.t3_logit, 1, logits, cap, n_out, stream, "logits");
    if (rc) return rc;
    return obj_field(c, OT_T3, event, c->E.t3_veto, 1, veto, cap, n_out, stream, "vetoes");
}

int lst_get_t5_features(lst_ctx *c, int32_t event, float *out, int64_t cap, int64_t *n_out,
                        void *stream)
{
    if (!c) return LST_E_INVALID;
    if (!c->features_valid) return fail(c, LST_E_STATE, "features have not been computed");
    return obj_field(c, OT_T5, event, c->E.t5_feat, 40, out, cap, n_out, stream, "feature rows");
}

// the pixel stage's device arrays, read back for one event's getters
struct PixRead {
    std::vector<int32_t> sorig, hlo, hup, slot, t5m[5], t3a, t3b, t3c;
    std::vector<int32_t> s5, o5, s3, o3, sev, sloc;
    std::vector<float> f5, f3;
    std::vector<uint8_t> k5, k3, clean, sk, keep;
    ShardCounts S;
};

static int pix_read(lst_ctx *c, void *stream, PixRead &R)
{
    if (c->stage < 8) return fail(c, LST_E_STATE, "the pixel stage has not run");
    int rc = sync_stream(c, stream);
    if (rc) return rc;
    const EvDev &E = c->E;
    ShardCounts &S = R.S;
    if ((rc = read_shards(c, S)) || (rc = check_fault(c, S.gc[GC_ERROR]))) return rc;
    if (S.gc[GC_OVERFLOW])
        return fail(c, LST_E_CAPACITY, "capacity overflow (mask %u)", S.gc[GC_OVERFLOW]);
    const uint32_t n5 = std::min<uint32_t>(S.gc[GC_PX5], (uint32_t)E.cap_pxc);
    const uint32_t n3 = std::min<uint32_t>(S.gc[GC_PX3], (uint32_t)E.cap_pxc);
    const int64_t n_sd = c->sd_off[c->n_events];
    const size_t nmd = S.span(OT_MD), nt3 = S.span(OT_T3), nt5 = S.span(OT_T5);
    if ((rc = sorted_orig(c, R.sorig, S.gc[GC_N_SORTED])) || (rc = d2h(c, R.hlo, E.md_hlo, nmd)) ||
        (rc = d2h(c, R.hup, E.md_hup, nmd)) || (rc = d2h(c, R.slot, E.md_slot, nmd)) ||
        (rc = d2h(c, R.t5m[0], E.t5_md0, nt5)) || (rc = d2h(c, R.t5m[1], E.t5_md1, nt5)) ||
        (rc = d2h(c, R.t5m[2], E.t5_md2, nt5)) || (rc = d2h(c, R.t5m[3], E.t5_md3, nt5)) ||
        (rc = d2h(c, R.t5m[4], E.t5_md4, nt5)) || (rc = d2h(c, R.t3a, E.t3_a, nt3)) ||
        (rc = d2h(c, R.t3b, E.t3_b, nt3)) || (rc = d2h(c, R.t3c, E.t3_c, nt3)) ||
        (rc = d2h(c, R.s5, E.c5_seed, n5)) || (rc = d2h(c, R.o5, E.c5_obj, n5)) ||
        (rc = d2h(c, R.f5, E.c5_score, n5)) || (rc = d2h(c, R.k5, E.c5_keep, n5)) ||
        (rc = d2h(c, R.s3, E.c3_seed, n3)) || (rc = d2h(c, R.o3, E.c3_obj, n3)) ||
        (rc = d2h(c, R.f3, E.c3_score, n3)) || (rc = d2h(c, R.k3, E.c3_keep, n3)) ||
        (rc = d2h(c, R.clean, E.t5_clean, nt5)) || (rc = d2h(c, R.keep, E.t5_keep, nt5)) ||
        (rc = d2h(c, R.sev, E.sd_ev, n_sd)) || (rc = d2h(c, R.sloc, E.sd_local, n_sd)) ||
        (rc = d2h(c, R.sk, E.sd_keep, n_sd)))
        return rc;
    R.s5.resize(n5); R.s3.resize(n3);
    return LST_OK;
}

// outer hit tuple (per-event indices) of a quintuplet (w 10) or triplet (w 6)
static void pix_tuple(const PixRead &R, int w, int32_t t, int32_t *out)
{
    for (int j = 0; j < w / 2; ++j) {
        const int32_t m = w == 10 ? R.t5m[j][t] : j == 0 ? R.t3a[t] : j == 1 ? R.t3b[t] : R.t3c[t];
        out[2 * j] = R.sorig[R.hlo[m]];
        out[2 * j + 1] = R.sorig[R.hup[m]];
    }
    for (int k = w; k < 10; ++k) out[k] = -1;
}

static int put_rows(lst_ctx *c, std::vector<std::array<int32_t, 13>> &rows, int width,
                    int32_t *out, int64_t cap, int64_t *n)
{
    std::sort(rows.begin(), rows.end());
    if (n) *n = (int64_t)rows.size();
    if ((int64_t)rows.size() > cap)
        return fail(c, LST_E_CAPACITY, "%lld rows, capacity %lld", (long long)rows.size(), (long long)cap);
    if (out)
        for (size_t i = 0; i < rows.size(); ++i)
            std::memcpy(&out[(size_t)width * i], rows[i].data(), sizeof(int32_t) * width);
    return LST_OK;
}

int lst_get_track_candidates(lst_ctx *c, int32_t event, int32_t *out, int64_t cap, int64_t *n,
                             void *stream)
{
    if (!c) return LST_E_INVALID;
    if (event < 0 || event >= c->n_events) return fail(c, LST_E_INVALID, "event %d", event);
    PixRead R;
    int rc = pix_read(c, stream, R);
    if (rc) return rc;
    std::vector<std::array<int32_t, 13>> rows;
    std::array<int32_t, 13> r{};
    for (size_t i = 0; i < R.s5.size(); ++i)
        if (R.k5[i] && R.sev[R.s5[i]] == event) {
            r[0] = LST_TC_PT5; r[1] = R.sloc[R.s5[i]];
            pix_tuple(R, 10, R.o5[i], &r[2]);
            rows.push_back(r);
        }
    for (size_t i = 0; i < R.s3.size(); ++i)
        if (R.k3[i] && R.sev[R.s3[i]] == event) {
            r[0] = LST_TC_PT3; r[1] = R.sloc[R.s3[i]];
            pix_tuple(R, 6, R.o3[i], &r[2]);
            rows.push_back(r);
        }
    const int lo_slot = event * c->n_mod, hi_slot = (event + 1) * c->n_mod;
    for (int sh = 0; sh < NSH; ++sh)
        for (uint32_t q = 0; q < R.S.n(OT_T5, sh); ++q) {
            const size_t t = (size_t)sh * R.S.rc[OT_T5] + q;
            const int32_t sl = R.slot[R.t5m[0][t]];
            if (!R.clean[t] || sl < lo_slot || sl >= hi_slot) continue;
            r[0] = LST_TC_T5; r[1] = -1;
            pix_tuple(R, 10, (int32_t)t, &r[2]);
            rows.push_back(r);
        }
    for (int32_t q = c->sd_off[event]; q < c->sd_off[event + 1]; ++q)
        if (R.sk[q]) {
            r[0] = LST_TC_PLS; r[1] = R.sloc[q];
            for (int k = 0; k < 10; ++k) r[2 + k] = -1;
            rows.push_back(r);
        }
    return put_rows(c, rows, 12, out, cap, n);
}

int lst_get_pixel_candidates(lst_ctx *c, int32_t event, int32_t what, int32_t *out, int64_t cap,
                             int64_t *n, void *stream)
{
    if (!c) return LST_E_INVALID;
    if (event < 0 || event >= c->n_events) return fail(c, LST_E_INVALID, "event %d", event);
    if (what != 0 && what != 1) return fail(c, LST_E_INVALID, "what %d (0 pT5, 1 pT3)", what);
    PixRead R;
    int rc = pix_read(c, stream, R);
    if (rc) return rc;
    const std::vector<int32_t> &sd = what ? R.s3 : R.s5, &ob = what ? R.o3 : R.o5;
    const std::vector<float> &sc = what ? R.f3 : R.f5;
    const std::vector<uint8_t> &kp = what ? R.k3 : R.k5;
    std::vector<std::array<int32_t, 13>> rows;
    std::array<int32_t, 13> r{};
    for (size_t i = 0; i < sd.size(); ++i) {
        if (R.sev[sd[i]] != event) continue;
        r[0] = R.sloc[sd[i]];
        pix_tuple(R, what ? 6 : 10, ob[i], &r[1]);
        std::memcpy(&r[11], &sc[i], sizeof(float));
        r[12] = kp[i];
        rows.push_back(r);
    }
    return put_rows(c, rows, 13, out, cap, n);
}

int lst_get_t3_features(lst_ctx *c, int32_t event, float *out, int64_t cap, int64_t *n_out,
                        void *stream)
{
    if (!c) return LST_E_INVALID;
    if (!c->t3_features_valid) return fail(c, LST_E_STATE, "features have not been computed");
    return obj_field(c, OT_T3, event, c->E.t3_feat, 40, out, cap, n_out, stream, "feature rows");
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner
// Order-independent checksum of everything the chain produced (all events):
// object counts per type and a sum of 64-bit mixes of every quintuplet's
// (event, hit tuple), separately for the kept ones.
static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdull; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ull; x ^= x >> 33;
    return x;
}

static int chain_checksum(lst_ctx *c, uint64_t *out)
{
    const EvDev &E = c->E;
    ShardCounts S;
    int rc = read_shards(c, S);
    if (rc) return rc;
    if (S.gc[GC_OVERFLOW] || S.gc[GC_ERROR] & 6)
        return fail(c, LST_E_CAPACITY, "tuning run overflowed or timed out (%u, %u)", S.gc[GC_OVERFLOW], S.gc[GC_ERROR]);
    std::vector<int32_t> sorig, hlo, hup, slot, m[5];
    std::vector<uint8_t> keep;
    if ((rc = sorted_orig(c, sorig, S.gc[GC_N_SORTED])) || (rc = d2h(c, hlo, E.md_hlo, S.span(OT_MD))) ||
        (rc = d2h(c, hup, E.md_hup, S.span(OT_MD))) || (rc = d2h(c, slot, E.md_slot, S.span(OT_MD))) ||
        (rc = d2h(c, keep, E.t5_keep, S.span(OT_T5))))
        return rc;
    int32_t *const dm[5] = {E.t5_md0, E.t5_md1, E.t5_md2, E.t5_md3, E.t5_md4};
    for (int j = 0; j < 5; ++j)
        if ((rc = d2h(c, m[j], (const int32_t *)dm[j], S.span(OT_T5)))) return rc;
    uint64_t h_all = 0, h_keep = 0;
    for (int sh = 0; sh < NSH; ++sh)
        for (uint32_t q = 0; q < S.n(OT_T5, sh); ++q) {
            const size_t t = (size_t)sh * S.rc[OT_T5] + q;
            uint64_t h = mix64((uint64_t)(slot[m[0][t]] / c->n_mod) + 0x9e3779b97f4a7c15ull);
            for (int j = 0; j < 5; ++j) {
                h = mix64(h ^ (uint64_t)(uint32_t)sorig[hlo[m[j][t]]]);
                h = mix64(h ^ (uint64_t)(uint32_t)sorig[hup[m[j][t]]]);
            }
            h_all += h;
            if (keep[t]) h_keep += h;
        }
    uint64_t h = 0;
    for (int t = 0; t < OT_COUNT; ++t) h = mix64(h ^ (uint64_t)S.stored(t));
    *out = mix64(h ^ h_all) ^ h_keep;
    return LST_OK;
}

// one eager chain with an event before and after every stage; per-stage us
static int timed_chain(lst_ctx *c, hipStream_t s, hipEvent_t *ev, double *stage_us)
{
    HIPCHK(c, hipEventRecord(ev[0], s));
    if (c->tune.persistent) {
        HIPCHK(c, launch_chain_persistent(c->E, c->M, c->K, c->zero_base, c->zero_bytes,
                                          c->tune.blocks_per_cu * c->n_cu, c->tune.lanes[ST_SEG],
                                          PERS_FULL, s));
        HIPCHK(c, hipEventRecord(ev[ST_COUNT], s));
    } else {
        const Tuning &t = c->tune;
        HIPCHK(c, launch_sort(c->E, c->M, t.grid[ST_SORT], sort_per_event(c), s));
        HIPCHK(c, hipEventRecord(ev[1], s));
        HIPCHK(c, launch_md(c->E, c->M, c->K, t.grid[ST_MD], t.lanes[ST_MD], s));
        HIPCHK(c, hipEventRecord(ev[2], s));
        HIPCHK(c, launch_seg(c->E, c->M, c->K, t.grid[ST_SEG], t.lanes[ST_SEG], seg_share(c), s));
        HIPCHK(c, hipEventRecord(ev[3], s));
        HIPCHK(c, launch_t3(c->E, c->M, c->K, t.grid[ST_T3], t.lanes[ST_T3], s));
        HIPCHK(c, hipEventRecord(ev[4], s));
        HIPCHK(c, launch_t5(c->E, c->M, c->K, t.grid[ST_T5], t.lanes[ST_T5], s));
        HIPCHK(c, hipEventRecord(ev[5], s));
        HIPCHK(c, launch_dedup(c->E, c->M, t.grid[ST_DEDUP], s));
        HIPCHK(c, hipEventRecord(ev[ST_COUNT], s));
    }
    HIPCHK(c, hipEventSynchronize(ev[ST_COUNT]));
    for (int i = 0; i < ST_COUNT; ++i) stage_us[i] = 0.0;
    float ms = 0.0f;
    if (c->tune.persistent) {
        HIPCHK(c, hipEventElapsedTime(&ms, ev[0], ev[ST_COUNT]));
        stage_us[0] = 1e3 * ms;
    } else {
        for (int i = 0; i < ST_COUNT; ++i) {
            HIPCHK(c, hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            stage_us[i] = 1e3 * ms;
        }
    }
    return LST_OK;
}

static double median(std::vector<double> v)
{
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

// median over `reps` chains of one stage's time (stage < 0: whole chain);
// the outputs of the last run must carry checksum `want`
static int measure(lst_ctx *c, hipStream_t s, hipEvent_t *ev, int reps, int stage,
                   uint64_t want, double *us, bool *valid)
{
    std::vector<double> v;
    double st[ST_COUNT];
    int rc;
    for (int r = 0; r <= reps; ++r) {
        if ((rc = timed_chain(c, s, ev, st))) return rc;
        double tot = 0.0;
        for (int i = 0; i < ST_COUNT; ++i) tot += st[i];
        if (r > 0) v.push_back(stage < 0 ? tot : st[stage]);
    }
    uint64_t h = 0;
    rc = chain_checksum(c, &h);
    *valid = rc == LST_OK && h == want;
    *us = median(v);
    return LST_OK;
}

static std::string tuning_key(const lst_ctx *c)
{
    char buf[160];
    snprintf(buf, sizeof(buf), "nmod=%d events=%d hits=%d cap_hits=%lld cu=%d", c->n_mod, c->n_events,
             c->hit_off.empty() ? 0 : c->hit_off.back(), (long long)c->caps.hits, c->n_cu);
    return buf;
}

extern "C" int lst_tune(lst_ctx *c, const char *cache_path, int32_t reps, double *report, void *stream)
{
    int rc = need_stage(c, 1, "lst_tune");
    if (rc) return rc;
    if (reps < 1) reps = 5;
    hipStream_t s = (hipStream_t)stream;
    const std::string key = tuning_key(c);
    // cached choice for this batch shape
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[1024];
            while (fgets(line, sizeof(line), f)) {
                const std::string ln(line);
                if (ln.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
                const size_t p = ln.find("\"tuning\": [");
                int32_t g[14];
                if (p != std::string::npos &&
                    sscanf(ln.c_str() + p + 11, "%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d",
                           &g[0], &g[1], &g[2], &g[3], &g[4], &g[5], &g[6], &g[7], &g[8], &g[9],
                           &g[10], &g[11], &g[12], &g[13]) == 14 &&
                    lst_set_tuning(c, g, g + 6, g[12], g[13]) == LST_OK) {
                    fclose(f);
                    if (report) report[0] = -1.0;  // taken from the cache
                    return LST_OK;
                }
            }
            fclose(f);
        }
    }
    hipEvent_t ev[ST_COUNT + 1];
    for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
    default_tuning(c);
    drop_graph(c);
    double st[ST_COUNT];
    uint64_t ref = 0;
    bool valid = false;
    double best_stage[ST_COUNT];
    if ((rc = timed_chain(c, s, ev, st)) || (rc = chain_checksum(c, &ref))) goto done;
    {
        static const int cand[ST_COUNT][6] = {
            {256, 512, 1024, 2048, 0, 0},        // sort
            {512, 1024, 2048, 4096, 0, 0},       // md
            {512, 1024, 2048, 4096, 8192, 0},    // seg
            {512, 1024, 2048, 4096, 8192, 0},    // t3
            {512, 1024, 2048, 4096, 8192, 0},    // t5
            {128, 256, 512, 1024, 2048, 0},      // dedup
        };
        static const int lane_cand[4] = {64, 32, 16, 8};
        for (int stg = 0; stg < ST_COUNT; ++stg) {
            const bool grouped = stg >= ST_MD && stg <= ST_T5;
            int best_g = c->tune.grid[stg], best_l = c->tune.lanes[stg];
            double best = 1e30;
            for (int li = 0; li < (grouped ? 4 : 1); ++li) {
                if (grouped) c->tune.lanes[stg] = lane_cand[li];
                for (int k = 0; k < 6 && cand[stg][k]; ++k) {
                    c->tune.grid[stg] = cand[stg][k];
                    double us;
                    if ((rc = measure(c, s, ev, reps, stg, ref, &us, &valid))) goto done;
                    if (!valid) {
                        rc = fail(c, LST_E_HIP, "stage %d with grid %d, lanes %d changed the results",
                                  stg, cand[stg][k], c->tune.lanes[stg]);
                        goto done;
                    }
                    if (us < best) {
                        best = us;
                        best_g = cand[stg][k];
                        best_l = c->tune.lanes[stg];
                    }
                }
            }
            c->tune.grid[stg] = best_g;
            c->tune.lanes[stg] = best_l;
            best_stage[stg] = best;
        }
        double graph_us = 0.0, pers_us = 1e30;
        if ((rc = measure(c, s, ev, reps, -1, ref, &graph_us, &valid))) goto done;
        // the persistent kernel runs the segment stage's group width everywhere
        const int occ = std::max(1, persistent_blocks_per_cu(c->tune.lanes[ST_SEG]));
        int best_bpc = 1;
        c->tune.persistent = 1;
        for (int bpc = 1; bpc <= occ; ++bpc) {
            c->tune.blocks_per_cu = bpc;
            double us;
            if ((rc = measure(c, s, ev, reps, -1, ref, &us, &valid))) goto done;
            if (valid && us < pers_us) { pers_us = us; best_bpc = bpc; }
        }
        c->tune.blocks_per_cu = best_bpc;
        c->tune.persistent = pers_us < graph_us ? 1 : 0;
        if (report) {
            for (int i = 0; i < ST_COUNT; ++i) report[i] = best_stage[i];
            report[ST_COUNT] = graph_us;
            report[ST_COUNT + 1] = pers_us;
        }
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (f) {
                const Tuning &t = c->tune;
                fprintf(f, "{\"key\": \"%s\", \"tuning\": [%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, "
                           "%d, %d, %d, %d], \"chain_us\": %.2f, \"persistent_us\": %.2f}\n",
                        key.c_str(), t.grid[0], t.grid[1], t.grid[2], t.grid[3], t.grid[4], t.grid[5],
                        t.lanes[0], t.lanes[1], t.lanes[2], t.lanes[3], t.lanes[4], t.lanes[5],
                        t.persistent, t.blocks_per_cu, graph_us, pers_us);
                fclose(f);
            }
        }
    }
done:
    for (auto &e : ev) (void)hipEventDestroy(e);
    drop_graph(c);
    c->counts_valid = false;
    c->stage = 7;
    return rc;
}
