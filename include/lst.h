/* lst.h -- C ABI of the MI355X Segment Linking (Line Segment Tracking) library.
 *
 * Method: arXiv:2209.13711, "Segment Linking: A Highly Parallelizable Track
 * Reconstruction Algorithm for HL-LHC".  The library runs the data-parallel,
 * module-local part of the method on one GPU: stubs (mini-doublets, Sec. 2),
 * segments, triplets and quintuplets built from every candidate combination
 * under geometric and kinematic requirements (Sec. 2.1), and removal of
 * quintuplets that share hits (Sec. 2.1, cross-cleaning rule that objects do
 * not share any hits).
 *
 * Conventions
 *  - Every function returns LST_OK (0) or a negative LST_E_* code; the message
 *    of the last failure is returned by lst_last_error.  Nothing throws.
 *  - Pointers are plain host or device pointers; the caller keeps ownership of
 *    everything it passes in (the library copies what it keeps).  Device
 *    memory for per-event work is the caller's arena (lst_attach_arena).
 *  - "stream" is a hipStream_t passed as void* (NULL = default stream).  Stage
 *    calls are asynchronous on it; kernel-side errors and capacity overflow
 *    surface at the next synchronising call (lst_get_counts / lst_get_objects).
 *  - A context is not thread safe; separate contexts are independent.
 *  - Output hit indices are the caller's per-event indices (position of the
 *    hit inside its event in the arrays given to lst_load_hits).  Tuples are
 *    in canonical order: mini-doublets inner to outer, each as (lower-sensor
 *    hit, upper-sensor hit).
 */
#ifndef LST_H
#define LST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LST_OK 0
#define LST_E_INVALID (-1)  /* bad argument or input value */
#define LST_E_STATE (-2)    /* call out of order (no geometry, no arena, no hits) */
#define LST_E_CAPACITY (-3) /* an output did not fit its capacity; counts report the need */
#define LST_E_HIP (-4)      /* HIP runtime error */
#define LST_E_NOMEM (-5)    /* host or device allocation failed */
#define LST_E_FAULT (-6)    /* a kernel-side wait timed out (error_flags bit 1 or 2):
                               the chain's outputs are unusable */

/* object kinds and their tuple widths (hit indices per object) */
enum lst_kind {
    LST_MD = 0,      /* width 2  */
    LST_SEG = 1,     /* width 4  */
    LST_T3 = 2,      /* width 6  */
    LST_T5 = 3,      /* width 10 */
    LST_T5_KEPT = 4  /* width 10: quintuplets surviving duplicate removal */
};

/* primary parameter vector (double), in this order.  The library derives
 * all of its FP32 constants from these values. */
enum lst_param {
    LST_P_BFIELD = 0, /* solenoid field, T (3.8) */
    LST_P_PTMIN,      /* threshold transverse momentum, GeV (0.8, Sec. 2) */
    LST_P_Z0MAX,      /* half length of the luminous region, cm */
    LST_P_SIGU,       /* hit resolution along the precise module axis, cm */
    LST_P_SIGV,       /* hit resolution along the coarse module axis, cm */
    LST_P_NSIG,       /* window half width in resolution units */
    LST_P_EPSK,       /* relative curvature margin above the threshold curvature */
    LST_P_EPSA,       /* curvature agreement slack, fraction of the threshold curvature */
    LST_P_D0MAX,      /* transverse impact parameter allowed by the beam-line cut, cm */
    LST_P_XRPHI,      /* r-phi chi2 limit of quintuplets (2 dof) */
    LST_P_XRZ,        /* r-z chi2 limit of quintuplets (3 dof) */
    LST_P_W,          /* window scale applied to every cut */
    LST_P_MAP_DPHI,   /* azimuthal margin of the module map, rad */
    LST_P_MAP_DL,     /* length margin of the module map, cm */
    LST_N_PARAMS
};

/* module table layout: module_f32 is [LST_MOD_NF][n_modules] float SoA with
 * rows cx cy cz ux uy uz vx vy vz wx wy wz hu hv gap rmin rmax zmin zmax phi dphi
 * (centre between the sensors; u precise axis, v coarse axis, w sensor normal
 * away from the interaction point; half sizes; sensor gap; extents of the
 * module in r, z and azimuth).  module_i32 is [LST_MOD_NI][n_modules] int SoA
 * with rows layer (barrel 1..6, +z disks 7..11, -z disks 12..16),
 * subdetector (0 barrel, 1 endcap), side (0, +1, -1), type (0 PS, 1 2S). */
#define LST_MOD_NF 21
#define LST_MOD_NI 4

/* chain modes (lst_set_mode) */
#define LST_MODE_CUTS 0 /* the plain cut chain */
#define LST_MODE_MLP 1  /* cut chain + learned veto of quintuplets before dedup */

/* learned scorer: inputs, and FP32 parameters in the order W1[64][40]
 * (row = hidden unit), b1[64], W2[64][64], b2[64], w3[64], b3 */
#define LST_MLP_NFEAT 40
#define LST_MLP_NPARAM 6849

typedef struct lst_ctx lst_ctx;

/* capacities of one arena (totals over all events of a batch) */
typedef struct {
    int32_t events; /* events per batch */
    int64_t hits;
    int64_t md;
    int64_t seg;
    int64_t t3;
    int64_t t5;
    int32_t features; /* nonzero: also hold the 40 scorer features per quintuplet */
    int64_t px_hits;  /* pixel hits (lst_load_pixel; 0: no pixel objects) */
    int64_t seeds;    /* pixel seeds (pLS) */
    int64_t px_cand;  /* link candidates of each kind (pT5, pT3) */
} lst_caps;

/* per-event result summary.  n_* are the numbers of objects and cand_* the
 * algorithmic candidate counts (pairs evaluated by each stage).  When a stage
 * ran out of capacity (LST_E_CAPACITY) the arrays are incomplete and every
 * event reports instead the batch-wide number of MD/SEG/T3/T5 required.  overflow_mask bit k = stage k (MD, SEG,
 * T3, T5) ran out of capacity; error_flags bit 0 = a hit with an invalid
 * module or sensor id was skipped, bit 1 = a persistent-chain barrier timed
 * out, bit 2 = the hit grouping failed: its scan timed out waiting for a
 * predecessor tile, or a hit's grouped position fell outside the hit arrays
 * (neither should ever happen).  With bit 1 or 2 set the outputs are unusable:
 * lst_get_counts fills *out (so the flags can be read) and returns
 * LST_E_FAULT, and every getter of objects, scores, logits or features
 * returns LST_E_FAULT; the bin counts are cleared so that the next chain
 * starts from a clean state. */
typedef struct {
    int64_t n_hits, n_md, n_seg, n_t3, n_t5, n_t5_kept;
    int64_t cand_md, cand_seg, cand_t3, cand_t5;
    int32_t overflow_mask, error_flags;
    int64_t dropped[4]; /* MD, SEG, T3, T5 removed by per-module capacities
                           (lst_set_capacities; 0 without them) */
    /* after lst_run_pixel: pixel seeds; pT5 link candidates and survivors;
     * pT3 link candidates and those left after cross-cleaning; track
     * candidates (pT5 + pT3 + T5 + pLS); 0 before */
    int64_t n_pls, cand_pt5, n_pt5, cand_pt3, n_pt3, n_tc;
    /* 1: the context was in scorer mode (LST_MODE_MLP) with no network
     * loaded, or with every loaded one rejected, so the batch ran the plain
     * cut chain; 0 otherwise */
    int32_t mlp_fallback;
} lst_counts;

/* Create a context on HIP device `device`.  params: LST_N_PARAMS doubles. */
int lst_create(lst_ctx **out, int device, const double *params, int32_t n_params);
void lst_destroy(lst_ctx *ctx);
const char *lst_last_error(const lst_ctx *ctx);

/* Load the detector description (host arrays, copied) and build the module
 * compatibility map (Sec. 2.1: modules on the next logical layer reachable by
 * +-q helices of threshold p_T from the luminous region).  Synchronous. */
int lst_load_geometry(lst_ctx *ctx, int32_t n_modules, const float *module_f32,
                      const int32_t *module_i32);

/* Stateless, host only (no device needed): the module map lst_load_geometry
 * would build for this geometry and parameter vector.  row_ptr [n_modules+1],
 * col [cap_col]; *n_edges is set even when cap_col is too small (then
 * LST_E_CAPACITY). */
int lst_build_map(const double *params, int32_t n_params, int32_t n_modules,
                  const float *module_f32, const int32_t *module_i32, int32_t *row_ptr,
                  int32_t *col, int64_t cap_col, int64_t *n_edges);

/* Copy the map out: row_ptr [n_modules+1], col [cap_col]; *n_edges is set even
 * when cap_col is too small (then LST_E_CAPACITY). */
int lst_get_map(lst_ctx *ctx, int32_t *row_ptr, int32_t *col, int64_t cap_col,
                int64_t *n_edges);

/* Device bytes an arena needs for the given capacities (geometry loaded). */
int lst_arena_bytes(const lst_ctx *ctx, const lst_caps *caps, size_t *bytes);

/* Hand the library a device buffer (e.g. a framework-allocated tensor) to
 * carve its per-event arrays from.  The caller keeps ownership and must keep
 * it alive while the context uses it. */
int lst_attach_arena(lst_ctx *ctx, void *dev_ptr, size_t bytes, const lst_caps *caps);

/* Load a batch of n_events events: hits of event e are [hit_offsets[e],
 * hit_offsets[e+1]) of x, y, z (cm), module (0..n_modules-1), sensor (0 lower,
 * 1 upper).  hit_offsets is a host array; the hit arrays are host pointers
 * (on_device = 0) or device pointers (on_device = 1).  Copies are enqueued on
 * `stream`; host arrays must stay valid until the stream reaches them. */
int lst_load_hits(lst_ctx *ctx, int32_t n_events, const int32_t *hit_offsets, const float *x,
                  const float *y, const float *z, const int32_t *module, const uint8_t *sensor,
                  int on_device, void *stream);

/* Half-precision hit storage (Sec. 4, Summary and Outlook: half-precision
 * data types).  fp16 = 1: the grouping stage stores each hit as its in-plane
 * coordinates in its module's frame, relative to the module centre (u along
 * the precise axis, v along the coarse one), each rounded to binary16
 * (nearest even), with its per-event index: 8 bytes instead of 16; the
 * mini-doublet stage rebuilds the FP32 position centre + u U + v V +
 * (+-gap/2) W (every operation FP32, in that order) and every later stage
 * works on it.  Module half-sizes are below 8 cm, so each coordinate moves by
 * at most 2^-9 cm.  fp16 = 0 (default): FP32 positions.  Later chains use the
 * mode; a batch grouped in the other mode must be grouped again
 * (LST_E_STATE until then).  LST_E_INVALID for other values. */
int lst_set_hit_storage(lst_ctx *ctx, int32_t fp16);

/* Per-module capacities (Sec. 3: every object kind held in arrays of a fixed
 * capacity per module, set at the 99.9 % or 99.99 % quantile of the
 * per-module occupancy, at a cost of 1-2 % in efficiency).  caps4 = the
 * capacity of MD, SEG, T3, T5 per module (0: none; NULL: all off), applied by
 * every later chain: right after a stage, a module (that of an object's first
 * mini-doublet) holding more objects of the stage's kind than its capacity
 * keeps the ones whose tuples of per-event hit indices are smallest
 * (lexicographic order) and the others are removed before the next stage
 * runs; lst_counts.dropped reports how many per kind.  The rule is
 * deterministic (the paper's GPU keeps whichever objects arrive first).  The
 * arrays stay compact: the mode reproduces the paper's selection, and the
 * memory its fixed per-module layout would take is caps x modules.  Runs
 * with the per-stage chain (lst_run_chain, lst_run_chain_graph); the
 * persistent kernel returns LST_E_STATE while capacities are set.
 * LST_E_INVALID for a negative capacity. */
int lst_set_capacities(lst_ctx *ctx, const int32_t *caps4);

/* Stages (asynchronous on `stream`), each requiring the previous one:
 * lst_run_sort      hits grouped by (event, module, sensor)
 * lst_run_md        mini-doublets (stubs), Sec. 2
 * lst_run_segments  segments over map edges, Sec. 2.1
 * lst_run_triplets  triplets: segment pairs sharing a mini-doublet, Sec. 2.1
 * lst_run_quintuplets quintuplets: triplet pairs sharing a mini-doublet, Sec. 2.1
 * lst_run_dedup     removal of quintuplets sharing hits (Sec. 2.1: objects
 *                   must not share hits): a quintuplet survives when, for each
 *                   of its hits, it has the smallest (score, hit tuple) key
 * lst_run_chain     all of the above in one call.
 * lst_run_sort may start a chain at any point after lst_load_hits; every
 * other stage runs exactly once, right after its predecessor (a repeated or
 * skipped stage returns LST_E_STATE and changes nothing). */
int lst_run_sort(lst_ctx *ctx, void *stream);
int lst_run_md(lst_ctx *ctx, void *stream);
int lst_run_segments(lst_ctx *ctx, void *stream);
int lst_run_triplets(lst_ctx *ctx, void *stream);
int lst_run_quintuplets(lst_ctx *ctx, void *stream);
int lst_run_dedup(lst_ctx *ctx, void *stream);
int lst_run_chain(lst_ctx *ctx, void *stream);

/* The same chain as lst_run_chain, launched as one hipGraph.  The graph is
 * captured on the first call after lst_attach_arena and replayed afterwards
 * for any batch that fits the arena (batch sizes are read on the device).
 * Results are identical to lst_run_chain. */
int lst_run_chain_graph(lst_ctx *ctx, void *stream);

/* Synchronise `stream`, then report event `event` (0..n_events-1).  Returns
 * LST_E_FAULT when a kernel-side wait timed out and LST_E_CAPACITY when any
 * stage overflowed (counts still filled in both cases). */
int lst_get_counts(lst_ctx *ctx, int32_t event, lst_counts *out, void *stream);

/* ---- pixel objects and track candidates (Sec. 2.1; kernel-flow figure of
 * Sec. 3) ------------------------------------------------------------------
 * Pixel parameters (double, in this order): pixel hit resolution across the
 * track and along z (cm); linking window (sine of the largest angle between
 * a pLS and an object it links to, times the window scale); squared eta-phi
 * distance under which cross-cleaning calls two objects duplicates; chi2
 * limits of pT5 (r-phi, r-z) and pT3 (r-phi, r-z). */
enum lst_pix_param {
    LST_PX_SIGRPHI = 0, LST_PX_SIGZ, LST_PX_WLINK, LST_PX_DR2, LST_PX_X5P, LST_PX_X5Z,
    LST_PX_X3P, LST_PX_X3Z, LST_PX_N_PARAMS
};
/* track-candidate types */
enum lst_tc_type { LST_TC_PT5 = 0, LST_TC_PT3 = 1, LST_TC_T5 = 2, LST_TC_PLS = 3 };

/* Pixel hits and seeds of the batch loaded by lst_load_hits (same n_events;
 * host arrays, copied, asynchronous on `stream` like lst_load_hits):
 * px_offsets[n_events + 1] first pixel hit of each event in x, y, z;
 * seed_offsets[n_events + 1] first seed of each event; seeds: four pixel hit
 * indices per seed, inner to outer, counted inside the seed's event.  A seed
 * index is its position inside its event.  Needs an arena whose caps hold
 * the pixel hits, seeds and link candidates (LST_E_CAPACITY otherwise);
 * LST_E_INVALID for a hit index outside its event or bad parameters. */
int lst_load_pixel(lst_ctx *ctx, int32_t n_events, const int32_t *px_offsets, const float *x,
                   const float *y, const float *z, const int32_t *seed_offsets,
                   const int32_t *seeds, const double *pix_params, int32_t n_pix_params,
                   void *stream);

/* The pixel stage after a whole chain (duplicate removal done) of the same
 * batch: each pLS linked to the kept quintuplets of its event (pT5) when
 * their directions lie inside the linking window and the chain of its four
 * pixel hits and five anchors passes the r-phi chi2 (circle through its
 * first hit and the 3rd and 5th anchors) and r-z chi2 (line in arc length)
 * cuts, score = their sum; inside the collection a pT5 survives iff no pT5
 * sharing one of its hits (pixel or outer) has a smaller (score, seed, hit
 * tuple) key.  The pLS no surviving pT5 uses link to the triplets (pT3, the
 * same way, circle through its first hit and the 1st and 3rd anchors).
 * Cross-cleaning in the paper's order: pT3 near a pT5 in eta-phi or sharing
 * a hit with one are duplicates; then kept quintuplets near or sharing a hit
 * with a pT5 or cleaned pT3; then the pLS used by neither, against all of
 * them, and among themselves the smaller seed index keeps a shared pixel
 * hit.  Asynchronous; per-stage chain, graph and persistent runs alike. */
int lst_run_pixel(lst_ctx *ctx, void *stream);

/* Track candidates of `event` (synchronises): 12 int32 per candidate: type
 * (lst_tc_type), seed index (-1 for T5), the outer hit tuple (10 hits for pT5
 * and T5, 6 for pT3, -1 padded).  *n set even when cap is too small
 * (LST_E_CAPACITY).  Order: pT5, pT3, T5, pLS. */
int lst_get_track_candidates(lst_ctx *ctx, int32_t event, int32_t *out12, int64_t cap,
                             int64_t *n, void *stream);

/* Link candidates of `event` (what 0: pT5, 1: pT3), 13 int32 each: seed,
 * outer hit tuple (-1 padded to 10), score bits, kept (pT5: survived the
 * collection's duplicate removal; pT3: also the cross-cleaning). */
int lst_get_pixel_candidates(lst_ctx *ctx, int32_t event, int32_t what, int32_t *out13,
                             int64_t cap, int64_t *n, void *stream);

/* Error-path hook for tests of the callers' handling of LST_E_FAULT: ORs
 * `bits` (error_flags bits 1 and 2 only) into the context's device error
 * word with a host-to-device copy after synchronising `stream`; no kernel
 * runs.  The next chain clears the word.  Needs a chain to have run. */
int lst_raise_error_flags(lst_ctx *ctx, int32_t bits, void *stream);

/* Synchronise `stream` and copy the objects of `kind` of `event` to out_host
 * (int32, width per lst_kind, capacity cap_tuples tuples).  *n_tuples is set
 * even when the capacity is too small (then LST_E_CAPACITY). */
int lst_get_objects(lst_ctx *ctx, int32_t event, int32_t kind, int32_t *out_host,
                    int64_t cap_tuples, int64_t *n_tuples, void *stream);

/* The 40 FP32 features of every stored quintuplet for the learned scorer
 * (asynchronous; needs an arena with caps.features set): per mini-doublet
 * r/100, z/100, bend pull, endcap flag, 2S flag; inner, outer and bridge
 * curvature over kappa_max; chi2/(1+chi2) in r-phi and r-z; r-phi pulls of
 * the 2nd and 4th anchors; r-z pulls of the 2nd to 4th; inner and outer
 * curvature agreement over its tolerance; r-z slope; lever arm/100; a
 * transverse impact parameter estimate.  lst_get_t5_features copies them
 * (40 per quintuplet, order of lst_get_objects(LST_T5)). */
int lst_run_t5_features(lst_ctx *ctx, void *stream);
int lst_get_t5_features(lst_ctx *ctx, int32_t event, float *out_host, int64_t cap_rows,
                        int64_t *n_rows, void *stream);

/* The 40 FP32 features of every stored triplet (22 used, the rest zero):
 * per mini-doublet r/100, z/100, bend pull, endcap flag, 2S flag; curvature
 * over kappa_max; each triplet cut's left-hand side over its limit (|k|,
 * signed k - k_origin, signed r-z residual); r-z slope; chord/100; an
 * impact-parameter estimate.  After lst_run_triplets; order of
 * lst_get_objects(LST_T3). */
int lst_run_t3_features(lst_ctx *ctx, void *stream);
int lst_get_t3_features(lst_ctx *ctx, int32_t event, float *out_host, int64_t cap_rows,
                        int64_t *n_rows, void *stream);

/* Quintuplet scores (chi2_rphi + chi2_rz) of `event`, in the order of
 * lst_get_objects(LST_T5). */
int lst_get_t5_scores(lst_ctx *ctx, int32_t event, float *out_host, int64_t cap,
                      int64_t *n, void *stream);

/* The whole chain as ONE persistent kernel: every stage runs inside a single
 * launch, separated by grid-wide barriers (release/acquire at device scope).
 * The grid is blocks_per_cu x compute units, bounded by the occupancy limit
 * so that every block is resident; a barrier that does not complete within
 * about half a second raises error_flags bit 1 and the kernel ends (no hang).
 * Results are identical to lst_run_chain.  lst_run_chain and
 * lst_run_chain_graph use this kernel when the tuning selects it. */
int lst_run_chain_persistent(lst_ctx *ctx, void *stream);

/* Launch shape: grid6 = blocks of 256 threads for the stages (hit grouping,
 * MD, segments, T3, T5, dedup); lanes6 = group width G (8, 16, 32 or 64;
 * used by MD, segments, T3, T5, ignored for the others; NULL keeps the
 * current values), which sets the inner objects a wave takes per round:
 * 64 / G module slots (MD) or inner MDs (segments), 256 / G inner MDs (T3,
 * T5); the wave walks their candidates together.  persistent = 1 runs the chain
 * as one persistent kernel of blocks_per_cu x CUs blocks, whose object
 * stages all use the segment stage's group width.  lst_get_tuning fills
 * out15 = grid6, lanes6, persistent, blocks_per_cu, number of CUs. */
int lst_set_tuning(lst_ctx *ctx, const int32_t *grid6, const int32_t *lanes6, int32_t persistent,
                   int32_t blocks_per_cu);
int lst_get_tuning(const lst_ctx *ctx, int32_t *out15);

/* Autotuner over the loaded batch: for each stage in turn, every candidate
 * grid (and, for the object stages, group width) is timed (median of `reps` chains, HIP events on `stream`) and its
 * outputs checksummed against the default launch shape (a candidate that
 * changes any object fails the call); then the persistent kernel is timed
 * for every co-resident blocks-per-CU value, and the faster of the per-stage
 * chain and the persistent chain is selected.  With cache_path, a choice
 * stored for the same batch shape is reused, and new choices are appended
 * (one JSON line each).  report (optional, 8 doubles): best per-stage us,
 * whole-chain us, persistent-chain us; report[0] = -1 when cached. */
int lst_tune(lst_ctx *ctx, const char *cache_path, int32_t reps, double *report, void *stream);

/* Project-written STREAM-like device copy (no context needed): dst = src for
 * n_bytes (a multiple of 16, 16-byte aligned device pointers), asynchronous
 * on `stream`.  Used to measure the achievable HBM bandwidth and to
 * calibrate the FETCH_SIZE / WRITE_SIZE counters against a known byte count. */
int lst_stream_copy(void *dst, const void *src, size_t n_bytes, void *stream);

/* ---- Learned quintuplet scorer --------------------------------------------
 * Not part of the paper.  Its outlook (Sec. 4, Summary and Outlook) plans to
 * revisit the object selection to raise efficiency and lower the fake rate;
 * this addition scores every quintuplet passing the cuts with a small network
 * and vetoes those it rejects before duplicate removal.  The cut chain stays
 * the fallback (LST_MODE_CUTS) and the reference for its efficiency and fake
 * rate.
 *
 * Network: 40 features -> 64 -> 64 -> 1 logit, ReLU after both hidden layers.
 * Features are standardised in FP32 as (f - mean) * istd and rounded to BF16
 * (nearest, ties to even); W1 and W2 are rounded to BF16 and the products
 * accumulated in FP32 on the matrix cores; the first hidden layer is rounded
 * to BF16 again before the second; w3, biases and the last layer are FP32.
 * A quintuplet is accepted iff logit >= threshold. */

/* Copy the scorer of `kind` (LST_T3: triplets, LST_T5: quintuplets; host
 * arrays: LST_MLP_NPARAM parameters, mean[40], istd[40]) and its logit
 * threshold into the context.  Synchronous; values must be finite: else
 * LST_E_INVALID, and the kind's earlier network, if any, is unloaded so that
 * its stage runs the plain cuts.  Each kind has its own network; either or
 * both may be loaded. */
int lst_mlp_load(lst_ctx *ctx, int32_t kind, const float *params, int32_t n_params,
                 const float *mean, const float *istd, float threshold);

/* LST_MODE_CUTS or LST_MODE_MLP.  In LST_MODE_MLP lst_run_chain,
 * lst_run_chain_graph and lst_run_chain_persistent include a scoring step
 * for every loaded kind: triplets are scored before the quintuplet stage (a
 * vetoed triplet joins no quintuplet), quintuplets before duplicate removal
 * (a vetoed quintuplet takes no part in it).  With no kind loaded (never
 * loaded, or rejected as not finite) the chain falls back to the plain cuts
 * and lst_counts.mlp_fallback reports it for every event of the batch. */
int lst_set_mode(lst_ctx *ctx, int32_t mode);

/* The scoring steps on their own (else LST_E_STATE): lst_run_t3_score
 * between lst_run_triplets and lst_run_quintuplets, lst_run_t5_score between
 * lst_run_quintuplets and lst_run_dedup.  Features are computed on the device
 * for every stored object, the logit stored, the veto set when logit <
 * threshold.  Asynchronous. */
int lst_run_t3_score(lst_ctx *ctx, void *stream);
int lst_run_t5_score(lst_ctx *ctx, void *stream);

/* Logits and vetoes (1 = rejected) of `event`'s quintuplets in the order of
 * lst_get_objects(LST_T5); host outputs of capacity cap.  Meaningful after a
 * scoring step. */
int lst_get_t5_logits(lst_ctx *ctx, int32_t event, float *logits_host, uint8_t *veto_host,
                      int64_t cap, int64_t *n, void *stream);
/* the same for triplets, in the order of lst_get_objects(LST_T3) */
int lst_get_t3_logits(lst_ctx *ctx, int32_t event, float *logits_host, uint8_t *veto_host,
                      int64_t cap, int64_t *n, void *stream);

/* ---- Training (device pointers, asynchronous on `stream`, ctx's device) ----
 * A batch of n rows: x [n][64] BF16 bit patterns (uint16; features 0..39
 * standardised, 40..63 zero), y [n] labels (0/1).  The loss is the mean
 * binary cross entropy on the logits; gradients flow through the BF16
 * roundings unchanged.  Every sum runs in a fixed order, so results are
 * bit-for-bit reproducible. */

/* device workspace lst_mlp_backward needs for n rows: 4 (n + 64 x
 * LST_MLP_NPARAM) bytes (per-row losses, partial gradients of up to 64 row
 * chunks) */
size_t lst_mlp_workspace_bytes(int64_t n);

/* x = BF16((feat - mean) * istd), zero padded to 64 columns; feat [n][40] FP32 */
int lst_mlp_prepare(lst_ctx *ctx, const float *feat, const float *mean, const float *istd,
                    int64_t n, uint16_t *x, void *stream);

/* logits [n] (FP32) of the network `params` (FP32 master weights, device).
 * h1 [n][64] (BF16 bits) and h2 [n][64] (FP32), the hidden activations, are
 * saved for lst_mlp_backward when both are non-null. */
int lst_mlp_forward(lst_ctx *ctx, const float *params, const uint16_t *x, int64_t n, float *logits,
                    uint16_t *h1, float *h2, void *stream);

/* grad [LST_MLP_NPARAM] = dL/dparams and *loss (device) for the batch whose
 * forward saved logits, h1, h2.  work: device scratch of work_bytes >=
 * lst_mlp_workspace_bytes(n) (else LST_E_CAPACITY). */
int lst_mlp_backward(lst_ctx *ctx, const float *params, const uint16_t *x, const uint8_t *y,
                     int64_t n, const float *logits, const uint16_t *h1, const float *h2,
                     void *work, size_t work_bytes, float *grad, float *loss, void *stream);

/* lst_mlp_backward without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid allocation).  The workspace is a
 * fixed device array inside the library, one per GPU, 1.8 MB, held from the
 * first lst_create on that GPU until the process ends; n at most 8192 rows
 * (else LST_E_CAPACITY, nothing launched).  The call allocates nothing and
 * gives the same results as lst_mlp_backward.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (different streams, threads or
 * contexts) race and must be ordered by the caller. */
int lst_mlp_backward_noalloc(lst_ctx *ctx, const float *params, const uint16_t *x,
                             const uint8_t *y, int64_t n, const float *logits, const uint16_t *h1,
                             const float *h2, float *grad, float *loss, void *stream);

/* One Adam step (bias corrected, step >= 1) on params with moments m, v
 * (device, LST_MLP_NPARAM each, updated in place). */
int lst_mlp_adam(lst_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t step,
                 float lr, float beta1, float beta2, float eps, void *stream);

/* n_steps Adam steps in one call.  Step i takes rows [order[i] * batch,
 * (order[i] + 1) * batch) of x [n_rows][64] and y [n_rows] through the
 * arithmetic of lst_mlp_forward, lst_mlp_backward (its loss into
 * losses[order[i]]) and lst_mlp_adam with step number first_step + 1 + i, in
 * the same order as those calls, hence the same results, in two launches per
 * step (the forward runs inside the gradient kernel, the Adam update inside
 * the chunk reduction) with no return to the caller between steps.  order:
 * host array of n_steps batch indices, each in 0 .. n_rows / batch - 1
 * (checked before anything is launched, else LST_E_INVALID).  logits, h1
 * and h2 are not used (kept for the signature; may be NULL).  Device
 * buffers: work (work_bytes >= lst_mlp_workspace_bytes(batch), else
 * LST_E_CAPACITY), grad, m, v [LST_MLP_NPARAM], losses [n_rows / batch].
 * Hyper-parameters as for lst_mlp_adam. */
int lst_mlp_train_steps(lst_ctx *ctx, float *params, const uint16_t *x, const uint8_t *y,
                        int64_t n_rows, int64_t batch, const int32_t *order, int32_t n_steps,
                        int32_t first_step, float *logits, uint16_t *h1, float *h2, void *work,
                        size_t work_bytes, float *grad, float *m, float *v, float *losses,
                        float lr, float beta1, float beta2, float eps, void *stream);

#ifdef __cplusplus
}
#endif
#endif
