// Internal layout shared by the host API and the kernels of liblst.
//
// Everything on the device is structure-of-arrays: one array per object
// property, so that consecutive lanes touch consecutive addresses (the SoA
// layout of Sec. 3 of the paper).  A batch of events is handled as one big
// detector with n_events x n_modules "slots": slot = event * n_modules + module,
// so a single event and a batch of 64 run the same kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lst {

// FP32 constants derived once from the primary parameter vector.
struct Consts {
    float kmax, klim, kh, tolu, tolv, tolkc, epsak;
    float z0max, sigu, sigv, nsig, d0max, w, w2, xrphi, xrz;
};

// Output reservation is spread over NSH counters per object type ("shards",
// chosen by blockIdx % NSH); shard s owns indices [s * rc, (s + 1) * rc) of
// the type's arrays, rc = ceil(capacity / NSH).  One hot counter would
// serialise every block's reservation across the chip.
constexpr int NSH = 32;
enum ObjType { OT_MD = 0, OT_SEG, OT_T3, OT_T5, OT_COUNT };

// Global counters (int32 / uint32).  Counters that many blocks update at
// once sit on their own 256-byte line: device-scope atomics on one line are
// serialised across the XCDs, so shard counters sharing a line would give
// no parallelism.
constexpr int GC_PAD = 64;   // uint32 stride of padded counters
enum GlobalCounter {
    GC_OVERFLOW = 0,   // bit k: object type k ran out of its region
    GC_ERROR,          // bit 0: invalid hit skipped
    GC_N_SORTED,       // number of grouped hits
    GC_TIEPOOL,        // entries taken from the dedup tie pool
    GC_SCAN,           // tile tickets of the look-back scan
    GC_DROP,           // [OT_COUNT] objects removed by per-module capacities
    GC_PX5 = GC_DROP + OT_COUNT,   // pT5 link candidates
    GC_PX3,            // pT3 link candidates
    GC_PXFREE,         // seeds that no kept pT5 uses (sd_free)
    GC_SH = GC_PAD     // [OT_COUNT][NSH] reservation shards, one line each
};
__host__ __device__ constexpr int gc_shard(int type, int s) { return GC_SH + (type * NSH + s) * GC_PAD; }
constexpr int GC_COUNT = GC_SH + OT_COUNT * NSH * GC_PAD;


// MI355X dispatches workgroup i to XCD i % 8, and each XCD has its own L2.
// Object stages split their work into NXCD azimuthal sectors and give
// sector x to the blocks with blockIdx % NXCD == x, so that the objects a
// block reads (its module's map neighbours) were mostly produced, and are
// still cached, on the same XCD.  Correctness never depends on the mapping.
constexpr int NXCD = 8;

struct ModDev {
    const float *cx, *cy, *cz, *ux, *uy, *uz, *vx, *vy, *vz, *g, *rl, *wx, *wy, *wz;
    const int32_t *barrel;   // 1 barrel, 0 endcap
    const int32_t *is2s;     // 1 for 2S modules
    const int32_t *map_ptr;  // [n_mod + 1]
    const int32_t *map_col;  // [n_edges]
    const int32_t *xorder;   // modules ordered by azimuthal sector, then layer
    int32_t sec_off[NXCD + 1];   // sector x = xorder[sec_off[x] .. sec_off[x + 1])
    int32_t n_mod;
};

// Batch descriptor, device resident so that a captured chain stays valid for
// any batch that fits the arena: [n_events, n_hits, n_slots, n_keys].
enum { D_NEV = 0, D_NHITS, D_NSLOTS, D_NKEYS, D_NPX, D_NSEEDS, D_COUNT };

struct EvDev {
    const int32_t *desc;             // [D_COUNT]
    int32_t cap_ev, cap_slots, cap_keys;
    int64_t cap_hits;
    uint32_t rc[OT_COUNT];           // region capacity per shard, per object type
    // inputs as loaded
    float *x, *y, *z;
    int32_t *module;
    uint8_t *sensor;
    int32_t *hit_off;        // [n_ev + 1]
    // grouping of hits by key = 2 * slot + sensor
    uint32_t *bcnt;          // [n_keys]     (zero between chains: the scan clears what it reads)
    uint32_t *hrank;         // [cap_hits]   each input hit's rank in its bin (histogram atomics)
    uint32_t *boff;          // [n_keys + 1]
    unsigned long long *scan_st;  // look-back scan: status per tile (zeroed at chain start)
    float4 *hsort;            // sorted hits: x, y, z and (int bits) the hit's per-event index
    // half-precision storage (half16 != 0): the sorted hits as module-local
    // (u, v) in binary16 (x: u | v << 16) and the per-event index (y)
    uint2 *hsort_h;
    int32_t half16;
    uint32_t *hmin;          // dedup: smallest quintuplet score bits per sorted hit
    int32_t *htie;           // dedup: how many quintuplets reach that score
    int32_t *hslot;          // dedup: [n_hits][TIE_SLOTS] quintuplets reaching it
    int32_t *thead;          // dedup: per hit, 1 + first pool entry of further ties (0: none)
    int32_t *tpool_t5, *tpool_next;  // dedup tie pool: quintuplet, 1 + next entry
    uint32_t cap_tpool;
    // mini-doublets
    int32_t *md_hlo, *md_hup, *md_slot;
    int4 *md_nbr;                    // module's first map edge, its edge count, event's first slot
    // anchor and window terms, three 16-byte records per MD so that a lane
    // gathers an MD with three loads: (x, y, z, r), (a, ca, 1/r, |sv|/r),
    // (dx, dy, |d|, sv)
    float4 *md_p0, *md_p1, *md_p2;
    float *md_bend;
    float *md_atol;                  // S3 bound w tol_u / |d| of the segment test
    uint8_t *md_bar;                 // bit 0: barrel module, bit 1: 2S module
    int32_t *md_start, *md_cnt;      // [n_slots]
    // segments (grouped by inner MD)
    int32_t *seg_in, *seg_out;
    int32_t *seg_start, *seg_cnt;    // [cap_md]
    // triplets (grouped by first MD)
    int32_t *t3_a, *t3_b, *t3_c;
    float *t3_k;
    int32_t *t3_start, *t3_cnt;      // [cap_md]
    uint8_t *t3_veto;                // 1: rejected by the learned scorer (no quintuplet uses it)
    float *t3_feat;                  // [span][40] features (learned scorer)
    float *t3_logit;                 // [span] scorer output
    // quintuplets (grouped by first MD)
    int32_t *t5_start, *t5_cnt;      // [cap_md]
    int32_t *t5_md0, *t5_md1, *t5_md2, *t5_md3, *t5_md4;
    float *t5_score;
    uint8_t *t5_keep;
    uint8_t *t5_veto;                // 1: rejected by the learned scorer
    int32_t *t5_hs, *t5_ho;          // dedup: [span][10] sorted and per-event hit indices
    float *t5_feat;                  // [span][40] features (learned scorer)
    float *t5_logit;                 // [span] scorer output
    // per-module capacities: drop flags (one byte per object, zero between
    // passes), each shard's prefix of kept objects (NSH x (largest rc + 1)),
    // objects removed per event and kind [cap_ev][OT_COUNT]
    uint8_t *cap_drop;
    int32_t *cap_pre;
    uint32_t *cap_nd;
    // pixel objects: pixel hits and seeds of the batch (pLS), object
    // directions, per-event lists, link candidates, cross-cleaning state
    int32_t cap_px, cap_seeds, cap_pxc;
    float *px_x, *px_y, *px_z;       // [cap_px]
    int32_t *px_off, *sd_off;        // [cap_ev + 1] first pixel hit / seed of each event
    int32_t *sd_hits;                // [cap_seeds][4] batch-wide pixel hit indices, inner to outer
    int32_t *sd_ev, *sd_local;       // [cap_seeds] event, index inside the event
    float4 *sd_dir;                  // [cap_seeds] tangent at the beam line, cot(theta)
    uint8_t *sd_used, *sd_keep;      // [cap_seeds] linked by a kept pT5/pT3; a track candidate
    float4 *t5_dir, *t3_dir;         // [span] directions of kept quintuplets, of triplets
    uint8_t *t5_clean;               // [span] kept quintuplet left after cross-cleaning
    // per-event lists (PXL_*), the kept quintuplets and the triplets also per
    // azimuth bin: counts, offsets, fill counters ([PXL_COUNT][cap_ev x PX_NB
    // + 1] each; a list's key is ev x PX_NB + bin, or ev), entries
    int32_t *pl_cnt, *pl_off, *pl_fill;
    int32_t *pl_k5, *pl_k3;          // kept quintuplets, triplets
    float4 *pl_k5d, *pl_k3d;         // their directions, in list order
    float4 *pl_d5, *pl_d3, *pl_dt;   // directions of kept pT5, cleaned pT3, cleaned T5
    // link candidates of pT5 (c5) and pT3 (c3): seed, object, score, kept
    int32_t *c5_seed, *c5_obj, *c3_seed, *c3_obj;   // [cap_pxc]
    float *c5_score, *c3_score;
    uint8_t *c5_keep, *c3_keep;
    int2 *sd_c5, *sd_c3;             // [cap_seeds] first candidate and count of each seed
    int32_t *sd_free;                // [cap_seeds] seeds that no kept pT5 uses
    unsigned long long *hmin_o;      // [cap_hits] smallest key per grouped outer hit
    unsigned long long *hmin_p;      // [cap_px]   smallest key per pixel hit
    uint8_t *hflag_o, *hflag_p;      // hits held by track candidates so far
    // counters (zeroed at chain start)
    uint32_t *gc;                    // [GC_COUNT]
    uint32_t *bar;                   // persistent-chain barrier counters [33]
};

constexpr int TIE_SLOTS = 8;
constexpr int BLOCK = 256;           // 4 waves of 64
constexpr int WAVES = BLOCK / 64;
constexpr int STAGE = 256;           // accepted objects a wave stages in LDS
constexpr int GRID_MAX = 2048;       // blocks of a grid-stride stage kernel
constexpr int SCAN_TILE = 4096;      // keys per tile of the look-back scan

// launchers (lst_kernels.hip)
hipError_t launch_copy(void *dst, const void *src, size_t n_bytes, hipStream_t s);
hipError_t launch_zero(const EvDev &E, void *zero_base, size_t zero_bytes, hipStream_t s);
// per_event: one block per (event, quarter of its bins), bins in LDS (batches)
hipError_t launch_sort(const EvDev &E, const ModDev &M, int grid, bool per_event, hipStream_t s);
size_t sort_ev_lds_bytes(int n_mod);
constexpr size_t SORT_EV_LDS_MAX = 160 * 1024;   // LDS of one gfx950 workgroup
constexpr int SORT_EV_MIN_EVENTS = 8;
hipError_t sort_ev_prepare(int n_mod);   // allows the per-event sort's LDS size
// lanes: width of the lane group that owns one inner object (8, 16, 32 or 64)
hipError_t launch_md(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                     hipStream_t s);
// share: the kernel whose runs of inner MDs of one module share their
// candidate enumeration when a wave takes consecutive MDs (batches); the
// other enumerates per MD (one event, whose one-pass order spreads the MDs)
hipError_t launch_seg(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                      bool share, hipStream_t s);
hipError_t launch_t3(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                     hipStream_t s);
hipError_t launch_t5(const EvDev &E, const ModDev &M, const Consts &K, int grid, int lanes,
                     hipStream_t s);
hipError_t launch_dedup(const EvDev &E, const ModDev &M, int grid, hipStream_t s);
// pixel objects (lst_pixel.hip)
enum { PXL_K5 = 0, PXL_K3, PXL_D5, PXL_D3, PXL_DT, PXL_COUNT };
constexpr int PX_NB = 64;   // azimuth bins of the per-event object lists
struct PixConsts {
    float sig2p, sigz, wl2, dr2, x5p, x5z, x3p, x3z;
    float wphi;   // azimuth half-range of the link window plus a margin (>= pi: all bins)
    float wdr;    // the same for the cross-cleaning closeness
};
hipError_t launch_pixel(const EvDev &E, const Consts &K, const PixConsts &P, hipStream_t s);
// per-module capacity `cap` of object type `type` (lst_cap.hip): objects of
// a module beyond it removed, the type's arrays compacted in place
hipError_t launch_cap(const EvDev &E, int type, int32_t cap, hipStream_t s);
// stop: PERS_FULL runs every stage; PERS_TO_T5 ends after the quintuplets,
// PERS_TO_T3 after the triplets (learned scoring follows as its own
// launches); lanes: group width of its four object stages
enum { PERS_FULL = 0, PERS_TO_T5 = 1, PERS_TO_T3 = 2 };
hipError_t launch_chain_persistent(const EvDev &E, const ModDev &M, const Consts &K,
                                   void *zero_base, size_t zero_bytes, int grid, int lanes,
                                   int stop, hipStream_t s);
int persistent_blocks_per_cu(int lanes);
hipError_t launch_t5_features(const EvDev &E, const Consts &K, int grid, hipStream_t s);
hipError_t launch_t3_features(const EvDev &E, const Consts &K, int grid, hipStream_t s);

// learned quintuplet scorer (lst_mlp.hip)
constexpr int MLP_NIN = 40, MLP_NH = 64;
constexpr int MLP_NPARAM = MLP_NH * MLP_NIN + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NH + 1;
size_t mlp_workspace_bytes(int64_t n);
hipError_t mlp_prepare(const float *F, const float *mean, const float *istd, int64_t n, uint16_t *X,
                       hipStream_t s);
hipError_t mlp_forward(const float *P, const uint16_t *X, int64_t n, float *logits, uint16_t *h1,
                       float *h2, hipStream_t s);
hipError_t mlp_backward(const float *P, const uint16_t *X, const uint8_t *y, int64_t n,
                        const float *logits, const uint16_t *h1, const float *h2, float *work,
                        float *grad, float *loss, hipStream_t s);
hipError_t mlp_adam(float *P, const float *grad, float *m, float *v, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s);
hipError_t mlp_train_step(float *P, const uint16_t *X, const uint8_t *y, int64_t n, float *work,
                          float *grad, float *loss, float *m, float *v, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t s);
// fixed backward workspace (no allocation): rows it holds, its size in floats
// (n loss rows + 64 chunks x MLP_NPARAM at n = MLP_FIXED_MAX_ROWS), and its
// device address on `device` (looked up once per device, then cached)
constexpr int64_t MLP_FIXED_MAX_ROWS = 8192;
constexpr size_t MLP_FIXED_SCRATCH_FLOATS = (size_t)MLP_FIXED_MAX_ROWS + (size_t)64 * MLP_NPARAM;
constexpr int MLP_FIXED_MAX_DEVICES = 64;
hipError_t mlp_fixed_scratch(int device, void **out);
// kind: OT_T3 or OT_T5
hipError_t mlp_score(const EvDev &E, const Consts &K, int kind, const float *P, const float *mean,
                     const float *istd, float threshold, int grid, hipStream_t s);

// Launch shape of every stage (blocks of BLOCK threads); chosen by the tuner.
enum StageId { ST_SORT = 0, ST_MD, ST_SEG, ST_T3, ST_T5, ST_DEDUP, ST_COUNT };
struct Tuning {
    int grid[ST_COUNT];
    int lanes[ST_COUNT];   // group width per stage (MD, SEG, T3, T5; others unused)
    int persistent;        // 1: the whole chain as one persistent kernel
    int blocks_per_cu;     // persistent grid = blocks_per_cu x CUs
};

}  // namespace lst
