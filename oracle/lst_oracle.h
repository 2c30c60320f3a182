/* CPU oracle of the Segment Linking hot path (arXiv:2209.13711).
 *
 * TEST INFRASTRUCTURE.  This is the slow, plain reference the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the library never does.  It shares no
 * source with the library: the geometry, the hits and the primary parameter
 * vector are its only common inputs.
 *
 * Stages, in the paper's order (Sec. 2.1 and the kernel-flow figure of
 * Sec. 3): compatibility map of modules -> mini-doublets (stubs) ->
 * segments -> triplets (T3) -> quintuplets (T5) -> removal of T5s that share
 * hits (Sec. 2.1, "objects do not share any hits").  Decisions are FP32; every
 * decision also gets its FP64 margin so that near-threshold cases can be told
 * apart from real disagreements.
 */
#ifndef LST_ORACLE_H
#define LST_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* primary parameters (double); the oracle derives its own FP32 constants */
enum {
    ORC_P_BFIELD = 0, /* T */
    ORC_P_PTMIN,      /* GeV, threshold p_T (0.8) */
    ORC_P_Z0MAX,      /* cm, luminous-region half length used by the pointing cuts */
    ORC_P_SIGU,       /* cm, precise-axis resolution */
    ORC_P_SIGV,       /* cm, coarse-axis resolution */
    ORC_P_NSIG,       /* window width in resolution units */
    ORC_P_EPSK,       /* relative curvature margin on the threshold */
    ORC_P_EPSA,       /* curvature agreement slack, fraction of kappa_max */
    ORC_P_D0MAX,      /* cm, transverse impact parameter allowed by the beam-line cut */
    ORC_P_XRPHI,      /* chi2 limit, r-phi, 2 dof */
    ORC_P_XRZ,        /* chi2 limit, r-z, 3 dof */
    ORC_P_W,          /* window scale */
    ORC_P_MAP_DPHI,   /* rad, azimuthal margin of the module map */
    ORC_P_MAP_DL,     /* cm, length margin of the module map */
    ORC_N_PARAMS
};

enum { ORC_MD = 0, ORC_SEG = 1, ORC_T3 = 2, ORC_T5 = 3, ORC_T5_KEPT = 4 };

typedef struct orc orc;

/* geometry: mod_f32 is [21][n_mod] float SoA, mod_i32 is [4][n_mod] int SoA
 * (layouts in synth/geometry.py).  Returns NULL on bad input. */
orc *orc_create(const double *params, int n_params, int n_mod, const float *mod_f32,
                const int32_t *mod_i32);
void orc_destroy(orc *o);

int64_t orc_map_edges(const orc *o);
void orc_map(const orc *o, int32_t *row_ptr, int32_t *col);

/* one event; hits in the caller's order (tuples refer to these indices) */
int orc_run(orc *o, int32_t n_hits, const float *x, const float *y, const float *z,
            const int32_t *module, const uint8_t *sensor);

int64_t orc_count(const orc *o, int kind);
/* tuples of kind (width 2, 4, 6, 10, 10) in caller hit indices */
void orc_tuples(const orc *o, int kind, int32_t *out);
/* algorithmic candidate counts: MD pairs, segment pairs, T3 pairs, T5 pairs */
void orc_cands(const orc *o, int64_t *out4);
void orc_t5_scores(const orc *o, float *out);
void orc_t5_keep(const orc *o, uint8_t *out);
void orc_t3_curv(const orc *o, float *out);
/* 40 FP32 features of every quintuplet / triplet, in the order of orc_tuples */
void orc_t5_features(const orc *o, float *out40);
void orc_t3_features(const orc *o, float *out40);
/* quintuplets and duplicate removal again on the stored triplets, with the
 * triplets whose t3_veto entry is set (orc_tuples(ORC_T3) order; NULL: none)
 * excluded from every quintuplet */
int orc_rerun_t5(orc *o, const uint8_t *t3_veto);

/* candidates whose FP64 margin is below 1e-5 (relative): tuple, margin and
 * the FP32 decision; kind 0..3 */
int64_t orc_near_count(const orc *o, int kind);
void orc_near(const orc *o, int kind, int32_t *tuples, double *margins, uint8_t *decision);

/* single-candidate evaluation for closed-form checks: each builds the MDs of
 * the given (module, lower hit, upper hit) triples without applying the MD
 * cut and fills `out` with the intermediate quantities listed in the source;
 * returns the FP32 decision */
int orc_eval_md(const orc *o, int module, const float *lo3, const float *up3, double *out);
int orc_eval_seg(const orc *o, const int32_t *mods2, const float *hits12, double *out);
int orc_eval_t3(const orc *o, const int32_t *mods3, const float *hits18, double *out);
int orc_eval_t5(const orc *o, const int32_t *mods5, const float *hits30, double *out);
int orc_eval_t3_features(const orc *o, const int32_t *mods3, const float *hits18, float *out40);
int orc_eval_t5_features(const orc *o, const int32_t *mods5, const float *hits30, float *out40);

/* FP64 decision margin of one candidate (kind ORC_MD..ORC_T5; ORC_MD takes one
 * module and six floats): relative distance to threshold of the cut that
 * decides it, infinite when two or more cuts fail */
double orc_eval_margin(const orc *o, int kind, const int32_t *mods, const float *hits);

/* Half-precision hit storage (Sec. 4 outlook): with fp16 set, every hit of
 * the next events is stored as its module-local in-plane coordinates (FP32
 * u, v relative to the module centre, each rounded to binary16, nearest
 * even) and rebuilt as centre + u U + v V + (sensor ? +g/2 : -g/2) W in FP32
 * before the chain runs on it.  orc_f32_to_f16 / orc_f16_to_f32: the
 * conversions it uses. */
void orc_set_hit_storage(orc *o, int fp16);
/* FP64 margins on (1, default) or off (0).  Off: the chain evaluates only
 * the FP32 instance of each cut; objects, candidates and scores are
 * unchanged and no near-threshold candidate is recorded. */
void orc_set_margins(orc *o, int on);
uint16_t orc_f32_to_f16(float f);
float orc_f16_to_f32(uint16_t h);

/* Per-module capacities (Sec. 3: fixed per-module output arrays truncated at
 * an occupancy quantile) of MD, SEG, T3, T5 (caps4; 0 or NULL: none), applied
 * from the next orc_run on: a module (that of an object's first MD) holding
 * more objects of a kind than its capacity keeps those with the smallest hit
 * tuples; later stages are built from the kept objects only.  orc_dropped:
 * objects removed per kind in the last event.  Returns -1 on a negative cap. */
int orc_set_truncation(orc *o, const int32_t *caps4);
void orc_dropped(const orc *o, int64_t *out4);

/* ---- pixel objects (Sec. 2.1; kernel-flow figure of Sec. 3) ----
 * Pixel parameter vector (double): pixel hit resolution across the track and
 * along z (cm), linking window (sine of the angle, scaled by the window scale
 * W), cross-cleaning distance (squared, eta-phi), chi2 limits of pT5 (r-phi
 * 6 dof, r-z 7 dof) and pT3 (r-phi 4 dof, r-z 5 dof). */
enum {
    ORC_PX_SIGRPHI = 0, ORC_PX_SIGZ, ORC_PX_WLINK, ORC_PX_DR2, ORC_PX_X5P, ORC_PX_X5Z,
    ORC_PX_X3P, ORC_PX_X3Z, ORC_PX_N_PARAMS
};
/* track-candidate types */
enum { ORC_TC_PT5 = 0, ORC_TC_PT3 = 1, ORC_TC_T5 = 2, ORC_TC_PLS = 3 };

/* pixel objects of the last orc_run: pixel hits (x, y, z, n_px) and seeds
 * (4 pixel hit indices each, inner to outer).  -1 on bad input or when no
 * event ran. */
int orc_run_pixel(orc *o, const double *pix_params, int n_pp, int32_t n_px, const float *x,
                  const float *y, const float *z, int32_t n_seeds, const int32_t *seeds);
/* what: 0 pT5 candidates, 1 surviving pT5, 2 pT3 candidates, 3 surviving
 * pT3 (after cross-cleaning), 4 track candidates, 5 near-threshold pixel
 * decisions */
int64_t orc_px_count(const orc *o, int what);
/* candidates (what 0: pT5, 2: pT3), 13 ints each: seed, 10 outer hits (-1
 * padded), score bits, survived the collection's duplicate removal */
void orc_px_candidates(const orc *o, int what, int32_t *out13);
/* track candidates, 12 ints each: type, seed (-1 for T5), 10 outer hits
 * (-1 padded) */
void orc_tc(const orc *o, int32_t *out12);

/* single pixel link for closed-form checks: pix12 = four pixel hits (x, y,
 * z), n_md = 5 or 3 MDs (mods, hits as for orc_eval_t5); out12: pLS tx, ty,
 * cot, object tx, ty, cot, window cos-term, sin^2, polar term, chi2_rphi,
 * chi2_rz, score; returns the FP32 decision (window and chi2 cuts) */
int orc_eval_link(const orc *o, const double *pix_params, const float *pix12, int n_md,
                  const int32_t *mods, const float *hits, double *out12);

/* derived FP32 constants (for inspection): kmax, klim, kh, tolu, tolv, tolkc, epsak */
void orc_consts(const orc *o, float *out7);

#ifdef __cplusplus
}
#endif
#endif
