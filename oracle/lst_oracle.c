/* CPU oracle of the Segment Linking hot path (arXiv:2209.13711).
 *
 * TEST INFRASTRUCTURE: plain, slow and single-threaded on purpose.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the HIP library never does, and the two share no source.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 *
 * What it computes, in the paper's order (Sec. 2.1, kernel-flow figure of
 * Sec. 3):
 *   1. the module compatibility map (modules on the next logical layer that
 *      a +-q helix of threshold p_T from the luminous region can reach),
 *   2. mini-doublets = stubs: every lower x upper hit pair of a module inside
 *      the window equivalent to p_T >= 0.8 GeV (Sec. 2),
 *   3. segments: every MD pair over every map edge, under the pointing,
 *      azimuthal-window and relative-angle requirements,
 *   4. triplets: every pair of segments sharing an MD,
 *   5. quintuplets: every pair of triplets sharing an MD, with a score,
 *   6. duplicate removal: a quintuplet is dropped when another one sharing at
 *      least one hit has a smaller (score, hit tuple) key (Sec. 2.1: objects
 *      must not share hits).
 * Every stage enumerates its full candidate space in nested loops.
 */
#define _DEFAULT_SOURCE
#include "lst_oracle.h"


#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ARC_A1 (1.0f / 6.0f)
#define ARC_A2 (3.0f / 40.0f)
#define ARC_A3 (5.0f / 112.0f)
#define ARC_A4 (35.0f / 1152.0f)
#define ARC_A5 (63.0f / 2816.0f)
#define ARC_A6 (231.0f / 13312.0f)

#define NEAR_REL 1e-5
#define LINK_MAXP 9     /* points of a linked chain: 4 pixel hits + 5 anchors */

/* ------------------------------------------------------------------------- */
typedef struct {
    float kmax, klim, kh, tolu, tolv, tolkc, epsak;
    float z0max, sigu, sigv, nsig, d0max, w, w2, xrphi, xrz;
} KCONST;

typedef struct {
    float cx, cy, cz, ux, uy, uz, vx, vy, vz, g, rl;
    int barrel;
    float wx, wy, wz;   /* sensor normal (hit storage rebuild) */
} MODF;

typedef struct {
    float x, y, z, r, a, ca, dx, dy, dn, bend, sv;
    int barrel, is2s, module, hlo, hup;
} MDREC;

typedef struct {
    int n;
    double lhs[8], rhs[8];
} CUTREC;

typedef struct {
    double kbr, resb, resd, pullb, pulld, zpull[3], chi2p, chi2z, score, tin, tout, sl, lae, kO;
} T5AUX;

typedef struct {
    double k, kO, dz, sl, lac, ra, rc, rhs[3];
} T3AUX;

/* float instance: the decisions */
#define R float
#define FN(name) name##_f
#define SQRT sqrtf
#define FABS fabsf
#define CUTS_FEATURES
#include "cuts.inc"
#undef CUTS_FEATURES
#undef R
#undef FN
#undef SQRT
#undef FABS

/* double instance: margins from the same float inputs */
#define R double
#define FN(name) name##_d
#define SQRT sqrt
#define FABS fabs
#include "cuts.inc"
#undef R
#undef FN
#undef SQRT
#undef FABS

/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t *v;
    int64_t n, cap;
} ivec;

static int iv_push(ivec *a, int32_t x)
{
    if (a->n == a->cap) {
        int64_t nc = a->cap ? 2 * a->cap : 1024;
        int32_t *p = (int32_t *)realloc(a->v, (size_t)nc * sizeof(int32_t));
        if (!p) return -1;
        a->v = p; a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

typedef struct {
    void *v;
    int64_t n, cap;
    size_t sz;
} gvec;

static void *gv_push(gvec *a)
{
    if (a->n == a->cap) {
        int64_t nc = a->cap ? 2 * a->cap : 1024;
        void *p = realloc(a->v, (size_t)nc * a->sz);
        if (!p) return NULL;
        a->v = p; a->cap = nc;
    }
    return (char *)a->v + (size_t)(a->n++) * a->sz;
}

static void gv_clear(gvec *a) { a->n = 0; }
static void gv_free(gvec *a) { free(a->v); a->v = NULL; a->n = a->cap = 0; }

typedef struct { int32_t i, o; } SEGREC;
typedef struct { int32_t a, b, c; float k; float feat[40]; } T3REC;
typedef struct { int32_t md[5]; float score; float feat[40]; } T5REC;
typedef struct { int32_t hits[10]; double margin; uint8_t decision; } NEARREC;
/* a pixel-linked candidate: seed (pLS), outer object (T5 or T3 index), score */
typedef struct { int32_t seed, obj; float score; } PXREC;
/* a track candidate: type (ORC_TC_*), seed or -1, outer hits (-1 padded) */
typedef struct { int32_t type, seed, hits[10]; } TCREC;

struct orc {
    KCONST K;
    int n_mod;
    MODF *mod;
    int32_t *layer, *subdet, *mtype;
    int32_t *map_ptr, *map_col;
    int64_t n_edges;
    /* event state */
    gvec md, seg, t3, t5, near[4];
    int32_t *seg_off, *t3_off;
    uint8_t *keep;
    uint8_t *t3_veto;   /* triplets excluded from the quintuplet stage (or NULL) */
    int32_t n_hits;
    int64_t cand[4];
    int hit_fp16;       /* hits stored as module-local FP16 (u, v) before the chain */
    int no_margin;      /* skip the FP64 instance (no near-threshold records) */
    int32_t cap[4];     /* per-module capacity of MD, SEG, T3, T5 (0: none) */
    int64_t dropped[4]; /* objects the capacities removed in the last event */
    /* pixel objects of the last orc_run_pixel */
    gvec pt5, pt3;      /* PXREC candidates */
    uint8_t *pt5_keep, *pt3_keep, *t5_clean, *pls_keep;
    int32_t *seeds;     /* copy of the last seeds (4 pixel hits each) */
    int32_t n_seeds, n_px;
    int64_t px_near;    /* pixel decisions within NEAR_REL of a threshold */
    gvec tc;            /* TCREC */
};

/* ------------------------------------------------------------------------- */
/* derived constants: computed once in FP64 from the primary parameters and
 * rounded once to FP32 */
static void derive_consts(const double *p, KCONST *K)
{
    double kmax = (0.0029979245800 * p[ORC_P_BFIELD]) / p[ORC_P_PTMIN];
    double klim = kmax * (1.0 + p[ORC_P_EPSK]);
    K->kmax = (float)kmax;
    K->klim = (float)klim;
    K->kh = (float)(0.5 * klim);
    K->tolu = (float)(p[ORC_P_NSIG] * sqrt(2.0) * p[ORC_P_SIGU]);
    K->tolv = (float)(p[ORC_P_NSIG] * sqrt(2.0) * p[ORC_P_SIGV]);
    K->tolkc = (float)(p[ORC_P_NSIG] * 8.0 * sqrt(1.5));
    K->epsak = (float)(p[ORC_P_EPSA] * kmax);
    K->z0max = (float)p[ORC_P_Z0MAX];
    K->sigu = (float)p[ORC_P_SIGU];
    K->sigv = (float)p[ORC_P_SIGV];
    K->nsig = (float)p[ORC_P_NSIG];
    K->d0max = (float)p[ORC_P_D0MAX];
    K->w = (float)p[ORC_P_W];
    K->w2 = (float)(p[ORC_P_W] * p[ORC_P_W]);
    K->xrphi = (float)p[ORC_P_XRPHI];
    K->xrz = (float)p[ORC_P_XRZ];
}

/* ------------------------------------------------------------------------- */
/* Module compatibility map (Sec. 2.1, CompModules figure): module B on the
 * next logical layer is linked to A when a helix of curvature up to the
 * threshold bound, starting on the beam line within the luminous region,
 * can pass through both.  Evaluated in FP64 over module extents:
 *   azimuth: |phi_B - phi_A| <= dphi_A + dphi_B + W (asin(rmax_B kh) -
 *            asin(rmin_A kh)) + margin;
 *   r-z:     straight lines from (0, +-W Z0) through the corners of A,
 *            extrapolated to B's radii (barrel) or disk plane (endcap), with
 *            the arc-over-chord factor of the threshold helix as slack. */
typedef struct {
    double rmin, rmax, zmin, zmax, phi, dphi, asn_lo, asn_hi, q;
    int layer, barrel, side;
} MODX;

static int next_layers(int layer, int *out)
{
    int n = 0;
    if (layer >= 1 && layer <= 6) {
        if (layer < 6) out[n++] = layer + 1;
        out[n++] = 7;
        out[n++] = 12;
    } else if ((layer >= 7 && layer <= 10) || (layer >= 12 && layer <= 15)) {
        out[n++] = layer + 1;
    }
    return n;
}

static int map_compatible(const MODX *A, const MODX *B, double w, double z0m, double mphi,
                          double mlen)
{
    if (B->rmax <= A->rmin) return 0;
    double Phi = (B->asn_hi - A->asn_lo) * w;
    double d = B->phi - A->phi;
    if (d > M_PI) d -= 2.0 * M_PI;
    if (d < -M_PI) d += 2.0 * M_PI;
    if (fabs(d) > ((A->dphi + B->dphi) + Phi) + mphi) return 0;
    if (B->barrel) {
        double tlo = B->rmin / A->rmax;
        double thi = (B->rmax / A->rmin) * B->q;
        double zlo = INFINITY, zhi = -INFINITY;
        double z0s[2] = {-z0m, z0m}, zs[2] = {A->zmin, A->zmax}, ts[2] = {tlo, thi};
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k) {
                    double zp = z0s[i] + (zs[j] - z0s[i]) * ts[k];
                    if (zp < zlo) zlo = zp;
                    if (zp > zhi) zhi = zp;
                }
        return (B->zmin <= zhi + mlen) && (B->zmax >= zlo - mlen);
    } else {
        double zlo_a = (B->side > 0) ? A->zmin : -A->zmax;
        double zhi_a = (B->side > 0) ? A->zmax : -A->zmin;
        double zd = fabs(B->zmin);
        if (zhi_a + z0m <= 0.0) return 0;
        double rlo = ((A->rmin * (zd + z0m)) / (zhi_a + z0m)) / B->q;
        double rhi = INFINITY;
        if (zlo_a - z0m > 0.0) rhi = (A->rmax * (zd - z0m)) / (zlo_a - z0m);
        return (B->rmin <= rhi + mlen) && (B->rmax >= rlo - mlen);
    }
}

static int build_map(orc *o, const double *p, const float *f32, const int32_t *i32)
{
    int n = o->n_mod;
    double kmax = (0.0029979245800 * p[ORC_P_BFIELD]) / p[ORC_P_PTMIN];
    double khm = 0.5 * kmax * (1.0 + p[ORC_P_EPSK]);
    double w = p[ORC_P_W];
    double z0m = p[ORC_P_Z0MAX] * w;
    MODX *X = (MODX *)calloc((size_t)n, sizeof(MODX));
    if (!X) return -1;
    for (int m = 0; m < n; ++m) {
        MODX *x = &X[m];
        x->rmin = f32[15 * n + m];
        x->rmax = f32[16 * n + m];
        x->zmin = f32[17 * n + m];
        x->zmax = f32[18 * n + m];
        x->phi = f32[19 * n + m];
        x->dphi = f32[20 * n + m];
        x->layer = i32[0 * n + m];
        x->barrel = i32[1 * n + m] == 0;
        x->side = i32[2 * n + m];
        double alo = x->rmin * khm, ahi = x->rmax * khm;
        if (alo > 1.0) alo = 1.0;
        if (ahi > 1.0) ahi = 1.0;
        x->asn_lo = asin(alo);
        x->asn_hi = asin(ahi);
        x->q = (ahi > 0.0) ? x->asn_hi / ahi : 1.0;
    }
    /* modules of each layer, in index order */
    int *lay_cnt = (int *)calloc(17, sizeof(int));
    int **lay_mods = (int **)calloc(17, sizeof(int *));
    for (int m = 0; m < n; ++m)
        if (X[m].layer >= 1 && X[m].layer <= 16) lay_cnt[X[m].layer]++;
    for (int l = 1; l <= 16; ++l) {
        lay_mods[l] = (int *)malloc((size_t)(lay_cnt[l] + 1) * sizeof(int));
        lay_cnt[l] = 0;
    }
    for (int m = 0; m < n; ++m)
        if (X[m].layer >= 1 && X[m].layer <= 16) lay_mods[X[m].layer][lay_cnt[X[m].layer]++] = m;
    ivec col = {0};
    o->map_ptr = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    o->map_ptr[0] = 0;
    for (int a = 0; a < n; ++a) {
        int nl[3];
        int nn = next_layers(X[a].layer, nl);
        /* candidate modules of all next layers, merged in increasing index */
        int cnt0 = (int)col.n;
        for (int t = 0; t < nn; ++t) {
            int L = nl[t];
            for (int j = 0; j < lay_cnt[L]; ++j) {
                int b = lay_mods[L][j];
                if (map_compatible(&X[a], &X[b], w, z0m, p[ORC_P_MAP_DPHI], p[ORC_P_MAP_DL]))
                    iv_push(&col, b);
            }
        }
        /* sort this row (insertion sort: rows are short) */
        for (int64_t i = cnt0 + 1; i < col.n; ++i) {
            int32_t key = col.v[i];
            int64_t j = i - 1;
            while (j >= cnt0 && col.v[j] > key) { col.v[j + 1] = col.v[j]; --j; }
            col.v[j + 1] = key;
        }
        o->map_ptr[a + 1] = (int32_t)col.n;
    }
    o->map_col = col.v;
    o->n_edges = col.n;
    for (int l = 1; l <= 16; ++l) free(lay_mods[l]);
    free(lay_mods);
    free(lay_cnt);
    free(X);
    return 0;
}

/* ------------------------------------------------------------------------- */
orc *orc_create(const double *params, int n_params, int n_mod, const float *f32,
                const int32_t *i32)
{
    if (!params || n_params < ORC_N_PARAMS || n_mod <= 0 || !f32 || !i32) return NULL;
    orc *o = (orc *)calloc(1, sizeof(orc));
    if (!o) return NULL;
    derive_consts(params, &o->K);
    o->n_mod = n_mod;
    o->mod = (MODF *)calloc((size_t)n_mod, sizeof(MODF));
    o->layer = (int32_t *)malloc((size_t)n_mod * sizeof(int32_t));
    o->subdet = (int32_t *)malloc((size_t)n_mod * sizeof(int32_t));
    o->mtype = (int32_t *)malloc((size_t)n_mod * sizeof(int32_t));
    for (int m = 0; m < n_mod; ++m) {
        MODF *M = &o->mod[m];
        M->cx = f32[0 * n_mod + m]; M->cy = f32[1 * n_mod + m]; M->cz = f32[2 * n_mod + m];
        M->ux = f32[3 * n_mod + m]; M->uy = f32[4 * n_mod + m]; M->uz = f32[5 * n_mod + m];
        M->vx = f32[6 * n_mod + m]; M->vy = f32[7 * n_mod + m]; M->vz = f32[8 * n_mod + m];
        float wx = f32[9 * n_mod + m], wy = f32[10 * n_mod + m];
        M->wx = wx; M->wy = wy; M->wz = f32[11 * n_mod + m];
        M->g = f32[14 * n_mod + m];
        M->barrel = i32[1 * n_mod + m] == 0;
        /* apothem of the lower sensor plane (barrel) */
        M->rl = ((M->cx * wx) + (M->cy * wy)) - (0.5f * M->g);
        o->layer[m] = i32[0 * n_mod + m];
        o->subdet[m] = i32[1 * n_mod + m];
        o->mtype[m] = i32[3 * n_mod + m];
    }
    o->md.sz = sizeof(MDREC);
    o->seg.sz = sizeof(SEGREC);
    o->t3.sz = sizeof(T3REC);
    o->t5.sz = sizeof(T5REC);
    for (int k = 0; k < 4; ++k) o->near[k].sz = sizeof(NEARREC);
    o->pt5.sz = sizeof(PXREC);
    o->pt3.sz = sizeof(PXREC);
    o->tc.sz = sizeof(TCREC);
    if (build_map(o, params, f32, i32) != 0) { orc_destroy(o); return NULL; }
    return o;
}

static void free_event(orc *o)
{
    free(o->seg_off); o->seg_off = NULL;
    free(o->t3_off); o->t3_off = NULL;
    free(o->keep); o->keep = NULL;
    free(o->t3_veto); o->t3_veto = NULL;
}

static void run_t5_dedup(orc *o);

void orc_destroy(orc *o)
{
    if (!o) return;
    free_event(o);
    gv_free(&o->md); gv_free(&o->seg); gv_free(&o->t3); gv_free(&o->t5);
    for (int k = 0; k < 4; ++k) gv_free(&o->near[k]);
    gv_free(&o->pt5); gv_free(&o->pt3); gv_free(&o->tc);
    free(o->pt5_keep); free(o->pt3_keep); free(o->t5_clean); free(o->pls_keep); free(o->seeds);
    free(o->mod); free(o->layer); free(o->subdet); free(o->mtype);
    free(o->map_ptr); free(o->map_col);
    free(o);
}

int64_t orc_map_edges(const orc *o) { return o->n_edges; }

void orc_map(const orc *o, int32_t *row_ptr, int32_t *col)
{
    memcpy(row_ptr, o->map_ptr, (size_t)(o->n_mod + 1) * sizeof(int32_t));
    memcpy(col, o->map_col, (size_t)o->n_edges * sizeof(int32_t));
}

void orc_consts(const orc *o, float *out)
{
    out[0] = o->K.kmax; out[1] = o->K.klim; out[2] = o->K.kh; out[3] = o->K.tolu;
    out[4] = o->K.tolv; out[5] = o->K.tolkc; out[6] = o->K.epsak;
}

/* ------------------------------------------------------------------------- */
/* decisive FP64 margin: the smallest relative distance to threshold of any
 * cut whose flip would flip the decision */
static double cut_margin(const CUTREC *f, const CUTREC *d)
{
    int nfail = 0, jfail = -1;
    for (int j = 0; j < f->n; ++j)
        if (!(f->lhs[j] <= f->rhs[j])) { nfail++; jfail = j; }
    double best = INFINITY;
    for (int j = 0; j < d->n; ++j) {
        if (nfail == 1 && j != jfail) continue;
        if (nfail > 1) break;
        double l = d->lhs[j], r = d->rhs[j];
        double s = fabs(l) > fabs(r) ? fabs(l) : fabs(r);
        if (s < 1e-30) s = 1e-30;
        double m = fabs(l - r) / s;
        if (isnan(m)) m = INFINITY;
        if (m < best) best = m;
    }
    return best;
}

static void md_hits(const orc *o, int32_t mdi, int32_t *h)
{
    const MDREC *m = &((const MDREC *)o->md.v)[mdi];
    h[0] = m->hlo; h[1] = m->hup;
}

static void push_near(orc *o, int kind, const int32_t *mds, int nmd, double margin, int dec)
{
    NEARREC *r = (NEARREC *)gv_push(&o->near[kind]);
    if (!r) return;
    memset(r->hits, 0xff, sizeof(r->hits));
    for (int j = 0; j < nmd; ++j) md_hits(o, mds[j], &r->hits[2 * j]);
    r->margin = margin;
    r->decision = (uint8_t)dec;
}

/* build an MD record from a hit pair without applying its cut */
static int make_md(const orc *o, int m, const float *L, const float *U, MDREC *md, CUTREC *cf,
                   CUTREC *cd)
{
    const MODF *M = &o->mod[m];
    float a, ca, r, bend, sv;
    double ad, cad, rd, bd, svd;
    int pass = md_cut_f(&o->K, M, L[0], L[1], L[2], U[0], U[1], U[2], cf, &a, &ca, &r, &bend, &sv);
    if (cd) md_cut_d(&o->K, M, L[0], L[1], L[2], U[0], U[1], U[2], cd, &ad, &cad, &rd, &bd, &svd);
    md->x = L[0]; md->y = L[1]; md->z = L[2];
    md->r = r; md->a = a; md->ca = ca; md->bend = bend; md->sv = sv;
    md->dx = U[0] - L[0];
    md->dy = U[1] - L[1];
    md->dn = sqrtf((md->dx * md->dx) + (md->dy * md->dy));
    md->barrel = M->barrel;
    md->is2s = o->mtype[m] == 1;
    md->module = m;
    return pass;
}


/* ------------------------------------------------------------------------- */
/* Per-module capacities (Sec. 3: every object kind lives in arrays of a fixed
 * capacity per module, set at a high quantile of the per-module occupancy, so
 * that a fuller module loses objects).  Which objects the paper's GPU loses
 * depends on thread timing; the rule here is fixed so that it can be
 * reproduced: a module holding more than `cap` objects of one kind keeps the
 * `cap` with the smallest tuples of caller hit indices (lexicographic), the
 * module of an object being that of its first mini-doublet.  keys: n rows of
 * w hit indices (all distinct); keep[i] = 1 iff fewer than cap rows are
 * smaller than row i.  Returns the number of rows dropped. */
static int64_t cap_keep(const int32_t *keys, int w, int64_t n, int64_t cap, uint8_t *keep)
{
    int64_t dropped = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t smaller = 0;
        for (int64_t j = 0; j < n; ++j) {
            int c = 0;   /* sign of (row j - row i) at the first differing hit */
            for (int k = 0; k < w && c == 0; ++k)
                c = (keys[j * w + k] > keys[i * w + k]) - (keys[j * w + k] < keys[i * w + k]);
            smaller += c < 0;
        }
        keep[i] = (uint8_t)(smaller < cap);
        dropped += !keep[i];
    }
    return dropped;
}

/* hit tuples of objects [lo, hi) of kind 1..3 (SEG, T3, T5) */
static int32_t *object_keys(const orc *o, int kind, int64_t lo, int64_t hi)
{
    const int w = kind == 1 ? 4 : kind == 2 ? 6 : 10;
    int32_t *k = (int32_t *)malloc((size_t)((hi - lo) > 0 ? (hi - lo) : 1) * w * sizeof(int32_t));
    for (int64_t i = lo; i < hi; ++i) {
        int32_t *r = &k[(i - lo) * w];
        if (kind == 1) {
            const SEGREC *S = &((const SEGREC *)o->seg.v)[i];
            md_hits(o, S->i, &r[0]); md_hits(o, S->o, &r[2]);
        } else if (kind == 2) {
            const T3REC *T = &((const T3REC *)o->t3.v)[i];
            md_hits(o, T->a, &r[0]); md_hits(o, T->b, &r[2]); md_hits(o, T->c, &r[4]);
        } else {
            const T5REC *T = &((const T5REC *)o->t5.v)[i];
            for (int j = 0; j < 5; ++j) md_hits(o, T->md[j], &r[2 * j]);
        }
    }
    return k;
}

/* Applies the capacity of `kind` (1..3) to objects grouped by inner MD:
 * off[md] .. off[md + 1] are the objects of MD md, md_off[m] .. md_off[m + 1]
 * the MDs of module m.  Compacts the kind's array in place (enumeration
 * order kept) and rewrites off. */
static void cap_grouped(orc *o, int kind, gvec *v, int32_t *off, const int32_t *md_off)
{
    const int64_t cap = o->cap[kind];
    if (cap <= 0) return;
    uint8_t *keep = (uint8_t *)malloc((size_t)(v->n > 0 ? v->n : 1));
    memset(keep, 1, (size_t)(v->n > 0 ? v->n : 1));
    for (int m = 0; m < o->n_mod; ++m) {
        const int64_t lo = off[md_off[m]], hi = off[md_off[m + 1]];
        if (hi - lo <= cap) continue;
        int32_t *keys = object_keys(o, kind, lo, hi);
        o->dropped[kind] += cap_keep(keys, kind == 1 ? 4 : 6, hi - lo, cap, &keep[lo]);
        free(keys);
    }
    const int64_t n_md = o->md.n;
    int64_t w = 0, r = 0;
    char *base = (char *)v->v;
    for (int64_t md = 0; md < n_md; ++md) {
        const int64_t end = off[md + 1];
        off[md] = (int32_t)w;
        for (; r < end; ++r)
            if (keep[r]) {
                if (w != r) memcpy(base + w * v->sz, base + r * v->sz, v->sz);
                ++w;
            }
    }
    off[n_md] = (int32_t)w;
    v->n = w;
    free(keep);
}

/* ---- half-precision hit storage (Sec. 4 outlook: half-precision data
 * types) ----
 * A hit is kept as its in-plane coordinates in its module's frame, relative
 * to the module centre, each rounded to binary16 (round to nearest, ties to
 * even), and its sensor; the chain then works on the FP32 position rebuilt
 * from them.  Every FP32 operation in the fixed order below. */

/* binary32 -> binary16 bits, round to nearest even (no NaN inputs here:
 * the coordinates are differences of finite positions) */
uint16_t orc_f32_to_f16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    const uint32_t sign = (u >> 16) & 0x8000u;
    const uint32_t a = u & 0x7fffffffu;
    if (a >= 0x7f800000u) return (uint16_t)(sign | 0x7c00u | (a > 0x7f800000u ? 0x200u : 0u));
    if (a >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);    /* rounds past 65504 */
    const int e = (int)(a >> 23) - 127;
    uint32_t mant = (a & 0x7fffffu) | 0x800000u;                 /* 24 bits, implicit one */
    int shift;                                                   /* bits dropped */
    uint32_t base;
    if (e >= -14) {                                              /* normal binary16 */
        shift = 13;
        base = ((uint32_t)(e + 15) << 10);
        mant &= 0x7fffffu;                                       /* fraction only */
        uint32_t q = mant >> shift, rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
        uint32_t r = base + q;
        if (rem > half || (rem == half && (q & 1u))) r += 1u;  /* carries into the exponent */
        return (uint16_t)(sign | r);
    }
    if (e < -25) return (uint16_t)sign;                          /* below half the smallest subnormal */
    shift = -e - 1;                                              /* subnormal: value = q 2^-24 */
    uint32_t q = mant >> shift, rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (q & 1u))) q += 1u;
    return (uint16_t)(sign | q);
}

float orc_f16_to_f32(uint16_t h)
{
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    const uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    float v;
    if (e == 0) {
        v = (float)m * 0x1p-24f;                                 /* exact: m < 2^10 */
    } else if (e == 31) {
        uint32_t u = sign | 0x7f800000u | (m << 13);
        memcpy(&v, &u, 4);
        return v;
    } else {
        uint32_t u = ((e + 112u) << 23) | (m << 13);
        memcpy(&v, &u, 4);
    }
    return sign ? -v : v;
}

/* the FP32 position a hit has after half-precision storage */
static void stored_hit(const MODF *M, int sensor, float x, float y, float z, float *out)
{
    float dx = x - M->cx, dy = y - M->cy, dz = z - M->cz;
    float u = ((dx * M->ux) + (dy * M->uy)) + (dz * M->uz);
    float v = ((dx * M->vx) + (dy * M->vy)) + (dz * M->vz);
    float uh = orc_f16_to_f32(orc_f32_to_f16(u));
    float vh = orc_f16_to_f32(orc_f32_to_f16(v));
    float w = (sensor ? 0.5f : -0.5f) * M->g;
    out[0] = ((M->cx + (uh * M->ux)) + (vh * M->vx)) + (w * M->wx);
    out[1] = ((M->cy + (uh * M->uy)) + (vh * M->vy)) + (w * M->wy);
    out[2] = ((M->cz + (uh * M->uz)) + (vh * M->vz)) + (w * M->wz);
}

void orc_set_hit_storage(orc *o, int fp16) { o->hit_fp16 = fp16 != 0; }

/* FP64 margins on (default) or off: off leaves every decision and object as
 * it is and records no near-threshold candidate; for timing the FP32
 * decisions alone */
void orc_set_margins(orc *o, int on) { o->no_margin = on == 0; }

int orc_set_truncation(orc *o, const int32_t *caps4)
{
    for (int k = 0; k < 4; ++k)
        if (caps4 && caps4[k] < 0) return -1;
    for (int k = 0; k < 4; ++k) o->cap[k] = caps4 ? caps4[k] : 0;
    return 0;
}

void orc_dropped(const orc *o, int64_t *out4) { memcpy(out4, o->dropped, sizeof(o->dropped)); }

int orc_run(orc *o, int32_t n_hits, const float *x, const float *y, const float *z,
            const int32_t *module, const uint8_t *sensor)
{
    if (n_hits < 0) return -1;
    for (int32_t h = 0; h < n_hits; ++h)
        if (module[h] < 0 || module[h] >= o->n_mod || sensor[h] > 1) return -1;
    float *xs = NULL, *ys = NULL, *zs = NULL;
    if (o->hit_fp16) {
        /* the chain runs on the positions half-precision storage gives back */
        xs = (float *)malloc((size_t)(n_hits > 0 ? n_hits : 1) * sizeof(float));
        ys = (float *)malloc((size_t)(n_hits > 0 ? n_hits : 1) * sizeof(float));
        zs = (float *)malloc((size_t)(n_hits > 0 ? n_hits : 1) * sizeof(float));
        for (int32_t h = 0; h < n_hits; ++h) {
            float p[3];
            stored_hit(&o->mod[module[h]], sensor[h], x[h], y[h], z[h], p);
            xs[h] = p[0]; ys[h] = p[1]; zs[h] = p[2];
        }
        x = xs; y = ys; z = zs;
    }
    free_event(o);
    gv_clear(&o->md); gv_clear(&o->seg); gv_clear(&o->t3); gv_clear(&o->t5);
    for (int k = 0; k < 4; ++k) gv_clear(&o->near[k]);
    memset(o->cand, 0, sizeof(o->cand));
    memset(o->dropped, 0, sizeof(o->dropped));
    int nm = o->n_mod;

    /* hits grouped by (module, sensor), original order kept inside a group */
    int64_t nb = 2 * (int64_t)nm;
    int32_t *boff = (int32_t *)calloc((size_t)(nb + 1), sizeof(int32_t));
    int32_t *bidx = (int32_t *)malloc((size_t)(n_hits > 0 ? n_hits : 1) * sizeof(int32_t));
    for (int32_t h = 0; h < n_hits; ++h) boff[2 * module[h] + sensor[h] + 1]++;
    for (int64_t b = 0; b < nb; ++b) boff[b + 1] += boff[b];
    int32_t *fill = (int32_t *)malloc((size_t)nb * sizeof(int32_t));
    memcpy(fill, boff, (size_t)nb * sizeof(int32_t));
    for (int32_t h = 0; h < n_hits; ++h) bidx[fill[2 * module[h] + sensor[h]]++] = h;
    free(fill);

    /* 1. mini-doublets, module by module */
    int32_t *md_off = (int32_t *)calloc((size_t)nm + 1, sizeof(int32_t));
    for (int m = 0; m < nm; ++m) {
        md_off[m] = (int32_t)o->md.n;
        for (int32_t i = boff[2 * m]; i < boff[2 * m + 1]; ++i) {
            for (int32_t j = boff[2 * m + 1]; j < boff[2 * m + 2]; ++j) {
                int32_t hl = bidx[i], hu = bidx[j];
                float L[3] = {x[hl], y[hl], z[hl]}, U[3] = {x[hu], y[hu], z[hu]};
                MDREC md;
                CUTREC cf, cd;
                o->cand[0]++;
                int pass = make_md(o, m, L, U, &md, &cf, o->no_margin ? NULL : &cd);
                md.hlo = hl; md.hup = hu;
                double mg = o->no_margin ? INFINITY : cut_margin(&cf, &cd);
                if (pass) *(MDREC *)gv_push(&o->md) = md;
                if (mg < NEAR_REL) {
                    NEARREC *r = (NEARREC *)gv_push(&o->near[0]);
                    memset(r->hits, 0xff, sizeof(r->hits));
                    r->hits[0] = hl; r->hits[1] = hu;
                    r->margin = mg; r->decision = (uint8_t)pass;
                }
            }
        }
        /* the module's MDs are enumerated in (lower, upper) hit order, so its
         * capacity keeps the first cap of them */
        if (o->cap[0] > 0 && o->md.n - md_off[m] > o->cap[0]) {
            o->dropped[0] += o->md.n - md_off[m] - o->cap[0];
            o->md.n = md_off[m] + o->cap[0];
        }
    }
    md_off[nm] = (int32_t)o->md.n;
    free(boff);
    free(bidx);
    const MDREC *MD = (const MDREC *)o->md.v;
    int64_t n_md = o->md.n;

    /* 2. segments: for each module A, each MD i of A, each map edge A->B,
     *    each MD o of B */
    o->seg_off = (int32_t *)calloc((size_t)n_md + 1, sizeof(int32_t));
    for (int a = 0; a < nm; ++a) {
        for (int32_t i = md_off[a]; i < md_off[a + 1]; ++i) {
            o->seg_off[i] = (int32_t)o->seg.n;
            for (int32_t e = o->map_ptr[a]; e < o->map_ptr[a + 1]; ++e) {
                int b = o->map_col[e];
                for (int32_t j = md_off[b]; j < md_off[b + 1]; ++j) {
                    CUTREC cf, cd;
                    float z0f, kOf;
                    double z0d, kOd;
                    o->cand[1]++;
                    int pass = seg_cut_f(&o->K, &MD[i], &MD[j], &cf, &z0f, &kOf);
                    if (!o->no_margin) seg_cut_d(&o->K, &MD[i], &MD[j], &cd, &z0d, &kOd);
                    if (pass) {
                        SEGREC *s = (SEGREC *)gv_push(&o->seg);
                        s->i = i; s->o = j;
                    }
                    double mg = o->no_margin ? INFINITY : cut_margin(&cf, &cd);
                    if (mg < NEAR_REL) {
                        int32_t mds[2] = {i, j};
                        push_near(o, 1, mds, 2, mg, pass);
                    }
                }
            }
        }
    }
    o->seg_off[n_md] = (int32_t)o->seg.n;
    cap_grouped(o, 1, &o->seg, o->seg_off, md_off);
    const SEGREC *SG = (const SEGREC *)o->seg.v;

    /* 3. triplets: segment (a->b) with every segment (b->c) */
    o->t3_off = (int32_t *)calloc((size_t)n_md + 1, sizeof(int32_t));
    {
        int64_t s = 0;
        for (int64_t a = 0; a < n_md; ++a) {
            o->t3_off[a] = (int32_t)o->t3.n;
            for (; s < o->seg_off[a + 1]; ++s) {
                int32_t b = SG[s].o;
                for (int32_t s2 = o->seg_off[b]; s2 < o->seg_off[b + 1]; ++s2) {
                    int32_t c = SG[s2].o;
                    CUTREC cf, cd;
                    float kf;
                    double kd;
                    o->cand[2]++;
                    T3AUX ax;
                    int pass = t3_cut_f(&o->K, &MD[a], &MD[b], &MD[c], &cf, &kf, &ax);
                    if (!o->no_margin) t3_cut_d(&o->K, &MD[a], &MD[b], &MD[c], &cd, &kd, NULL);
                    if (pass) {
                        T3REC *t = (T3REC *)gv_push(&o->t3);
                        t->a = (int32_t)a; t->b = b; t->c = c; t->k = kf;
                        const MDREC *P3[3] = {&MD[a], &MD[b], &MD[c]};
                        t3_features_f(&o->K, P3, &ax, t->feat);
                    }
                    double mg = o->no_margin ? INFINITY : cut_margin(&cf, &cd);
                    if (mg < NEAR_REL) {
                        int32_t mds[3] = {(int32_t)a, b, c};
                        push_near(o, 2, mds, 3, mg, pass);
                    }
                }
            }
        }
        o->t3_off[n_md] = (int32_t)o->t3.n;
    }
    cap_grouped(o, 2, &o->t3, o->t3_off, md_off);
    free(md_off);
    o->n_hits = n_hits;
    run_t5_dedup(o);
    free(xs); free(ys); free(zs);
    return 0;
}

/* 4. quintuplets and 5. duplicate removal, on the stored triplets; a
 * triplet with t3_veto set takes no part in any quintuplet */
static void run_t5_dedup(orc *o)
{
    const MDREC *MD = (const MDREC *)o->md.v;
    const int32_t n_hits = o->n_hits;
    gv_clear(&o->t5);
    gv_clear(&o->near[3]);
    o->cand[3] = 0;
    o->dropped[3] = 0;
    free(o->keep); o->keep = NULL;
    const T3REC *T3 = (const T3REC *)o->t3.v;

    /* 4. quintuplets: triplet (a,b,c) with every triplet (c,d,e) */
    for (int64_t t = 0; t < o->t3.n; ++t) {
        int32_t c = T3[t].c;
        for (int32_t t2 = o->t3_off[c]; t2 < o->t3_off[c + 1]; ++t2) {
            const MDREC *P[5] = {&MD[T3[t].a], &MD[T3[t].b], &MD[c], &MD[T3[t2].b],
                                 &MD[T3[t2].c]};
            if (o->t3_veto && (o->t3_veto[t] || o->t3_veto[t2])) {
                o->cand[3]++;   /* still a candidate pair of the stage */
                continue;
            }
            CUTREC cf, cd;
            T5AUX af, ad;
            o->cand[3]++;
            int pass = t5_cut_f(&o->K, P, T3[t].k, T3[t2].k, &cf, &af);
            if (!o->no_margin) t5_cut_d(&o->K, P, T3[t].k, T3[t2].k, &cd, &ad);
            int32_t mds[5] = {T3[t].a, T3[t].b, c, T3[t2].b, T3[t2].c};
            if (pass) {
                T5REC *q = (T5REC *)gv_push(&o->t5);
                memcpy(q->md, mds, sizeof(mds));
                q->score = (float)af.score;
                t5_features_f(&o->K, P, T3[t].k, T3[t2].k, &af, q->feat);
            }
            double mg = o->no_margin ? INFINITY : cut_margin(&cf, &cd);
            if (mg < NEAR_REL) push_near(o, 3, mds, 5, mg, pass);
        }
    }

    /* capacity per module of the first MD: the quintuplets come grouped by
     * their first triplet, hence by first MD and by its module */
    if (o->cap[3] > 0 && o->t5.n > 0) {
        T5REC *Q = (T5REC *)o->t5.v;
        uint8_t *keep = (uint8_t *)malloc((size_t)o->t5.n);
        int64_t lo = 0;
        while (lo < o->t5.n) {
            const int m = MD[Q[lo].md[0]].module;
            int64_t hi = lo + 1;
            while (hi < o->t5.n && MD[Q[hi].md[0]].module == m) ++hi;
            memset(&keep[lo], 1, (size_t)(hi - lo));
            if (hi - lo > o->cap[3]) {
                int32_t *keys = object_keys(o, 3, lo, hi);
                o->dropped[3] += cap_keep(keys, 10, hi - lo, o->cap[3], &keep[lo]);
                free(keys);
            }
            lo = hi;
        }
        int64_t w = 0;
        for (int64_t r = 0; r < o->t5.n; ++r)
            if (keep[r]) {
                if (w != r) Q[w] = Q[r];
                ++w;
            }
        o->t5.n = w;
        free(keep);
    }

    /* 5. duplicate removal over shared hits */
    int64_t n5 = o->t5.n;
    const T5REC *T5 = (const T5REC *)o->t5.v;
    o->keep = (uint8_t *)malloc((size_t)(n5 > 0 ? n5 : 1));
    int32_t *tup = (int32_t *)malloc((size_t)(n5 > 0 ? n5 : 1) * 10 * sizeof(int32_t));
    for (int64_t t = 0; t < n5; ++t)
        for (int j = 0; j < 5; ++j) md_hits(o, T5[t].md[j], &tup[t * 10 + 2 * j]);
    int32_t *hoff = (int32_t *)calloc((size_t)n_hits + 1, sizeof(int32_t));
    for (int64_t t = 0; t < n5 * 10; ++t) hoff[tup[t] + 1]++;
    for (int32_t h = 0; h < n_hits; ++h) hoff[h + 1] += hoff[h];
    int32_t *hcur = (int32_t *)malloc((size_t)(n_hits > 0 ? n_hits : 1) * sizeof(int32_t));
    memcpy(hcur, hoff, (size_t)n_hits * sizeof(int32_t));
    int32_t *hlist = (int32_t *)malloc((size_t)(n5 > 0 ? n5 * 10 : 1) * sizeof(int32_t));
    for (int64_t t = 0; t < n5; ++t)
        for (int j = 0; j < 10; ++j) hlist[hcur[tup[t * 10 + j]]++] = (int32_t)t;
    for (int64_t t = 0; t < n5; ++t) {
        int removed = 0;
        for (int j = 0; j < 10 && !removed; ++j) {
            int32_t h = tup[t * 10 + j];
            for (int32_t q = hoff[h]; q < hoff[h + 1] && !removed; ++q) {
                int32_t u = hlist[q];
                if (u == t) continue;
                int less = 0;
                if (T5[u].score < T5[t].score) less = 1;
                else if (T5[u].score == T5[t].score) {
                    for (int k = 0; k < 10; ++k) {
                        if (tup[u * 10 + k] != tup[t * 10 + k]) {
                            less = tup[u * 10 + k] < tup[t * 10 + k];
                            break;
                        }
                    }
                }
                if (less) removed = 1;
            }
        }
        o->keep[t] = (uint8_t)!removed;
    }
    free(tup); free(hoff); free(hcur); free(hlist);
}

/* ------------------------------------------------------------------------- */
int64_t orc_count(const orc *o, int kind)
{
    switch (kind) {
    case ORC_MD: return o->md.n;
    case ORC_SEG: return o->seg.n;
    case ORC_T3: return o->t3.n;
    case ORC_T5: return o->t5.n;
    case ORC_T5_KEPT: {
        int64_t c = 0;
        for (int64_t t = 0; t < o->t5.n; ++t) c += o->keep[t];
        return c;
    }
    }
    return -1;
}

void orc_tuples(const orc *o, int kind, int32_t *out)
{
    const SEGREC *SG = (const SEGREC *)o->seg.v;
    const T3REC *T3 = (const T3REC *)o->t3.v;
    const T5REC *T5 = (const T5REC *)o->t5.v;
    int64_t w = 0;
    switch (kind) {
    case ORC_MD:
        for (int64_t i = 0; i < o->md.n; ++i) md_hits(o, (int32_t)i, &out[2 * i]);
        break;
    case ORC_SEG:
        for (int64_t i = 0; i < o->seg.n; ++i) {
            md_hits(o, SG[i].i, &out[4 * i]);
            md_hits(o, SG[i].o, &out[4 * i + 2]);
        }
        break;
    case ORC_T3:
        for (int64_t i = 0; i < o->t3.n; ++i) {
            md_hits(o, T3[i].a, &out[6 * i]);
            md_hits(o, T3[i].b, &out[6 * i + 2]);
            md_hits(o, T3[i].c, &out[6 * i + 4]);
        }
        break;
    case ORC_T5:
    case ORC_T5_KEPT:
        for (int64_t i = 0; i < o->t5.n; ++i) {
            if (kind == ORC_T5_KEPT && !o->keep[i]) continue;
            for (int j = 0; j < 5; ++j) md_hits(o, T5[i].md[j], &out[10 * w + 2 * j]);
            w++;
        }
        break;
    }
}

void orc_cands(const orc *o, int64_t *out4) { memcpy(out4, o->cand, sizeof(o->cand)); }

void orc_t5_scores(const orc *o, float *out)
{
    const T5REC *T5 = (const T5REC *)o->t5.v;
    for (int64_t i = 0; i < o->t5.n; ++i) out[i] = T5[i].score;
}

void orc_t5_keep(const orc *o, uint8_t *out) { memcpy(out, o->keep, (size_t)o->t5.n); }

void orc_t5_features(const orc *o, float *out)
{
    const T5REC *T5 = (const T5REC *)o->t5.v;
    for (int64_t i = 0; i < o->t5.n; ++i) memcpy(&out[40 * i], T5[i].feat, sizeof(T5[i].feat));
}

void orc_t3_features(const orc *o, float *out)
{
    const T3REC *T3 = (const T3REC *)o->t3.v;
    for (int64_t i = 0; i < o->t3.n; ++i) memcpy(&out[40 * i], T3[i].feat, sizeof(T3[i].feat));
}

int orc_rerun_t5(orc *o, const uint8_t *t3_veto)
{
    if (!o->t3_off) return -1;
    free(o->t3_veto);
    o->t3_veto = NULL;
    if (t3_veto) {
        o->t3_veto = (uint8_t *)malloc((size_t)(o->t3.n > 0 ? o->t3.n : 1));
        if (!o->t3_veto) return -1;
        memcpy(o->t3_veto, t3_veto, (size_t)o->t3.n);
    }
    run_t5_dedup(o);
    return 0;
}

void orc_t3_curv(const orc *o, float *out)
{
    const T3REC *T3 = (const T3REC *)o->t3.v;
    for (int64_t i = 0; i < o->t3.n; ++i) out[i] = T3[i].k;
}

int64_t orc_near_count(const orc *o, int kind)
{
    return (kind >= 0 && kind < 4) ? o->near[kind].n : -1;
}

void orc_near(const orc *o, int kind, int32_t *tuples, double *margins, uint8_t *decision)
{
    static const int width[4] = {2, 4, 6, 10};
    const NEARREC *r = (const NEARREC *)o->near[kind].v;
    for (int64_t i = 0; i < o->near[kind].n; ++i) {
        memcpy(&tuples[i * width[kind]], r[i].hits, (size_t)width[kind] * sizeof(int32_t));
        margins[i] = r[i].margin;
        decision[i] = r[i].decision;
    }
}

/* ------------------------------------------------------------------------- */
/* orc_eval_md out: [|du-c0|, W h0, |dv-zc|, W hz, bend, a, ca, r] */
int orc_eval_md(const orc *o, int module, const float *lo3, const float *up3, double *out)
{
    MDREC md;
    CUTREC cf;
    int pass = make_md(o, module, lo3, up3, &md, &cf, NULL);
    out[0] = cf.lhs[0]; out[1] = cf.rhs[0]; out[2] = cf.lhs[1]; out[3] = cf.rhs[1];
    out[4] = md.bend; out[5] = md.a; out[6] = md.ca; out[7] = md.r;
    return pass;
}

static void eval_mds(const orc *o, int n, const int32_t *mods, const float *hits, MDREC *md)
{
    for (int j = 0; j < n; ++j) {
        CUTREC cf;
        make_md(o, mods[j], &hits[6 * j], &hits[6 * j + 3], &md[j], &cf, NULL);
    }
}

/* orc_eval_seg out: [lhs/rhs pairs of S2(cos), S2(sin), S1, S3 inner, S3 outer (0 when
 * absent)], then z0, kO, number of cuts */
int orc_eval_seg(const orc *o, const int32_t *mods2, const float *hits12, double *out)
{
    MDREC md[2];
    eval_mds(o, 2, mods2, hits12, md);
    CUTREC cf;
    float z0, kO;
    int pass = seg_cut_f(&o->K, &md[0], &md[1], &cf, &z0, &kO);
    for (int j = 0; j < 10; ++j) out[j] = 0.0;
    int p = 0;
    out[p++] = cf.lhs[0]; out[p++] = cf.rhs[0];
    out[p++] = cf.lhs[1]; out[p++] = cf.rhs[1];
    out[p++] = cf.lhs[2]; out[p++] = cf.rhs[2];
    int j = 3;
    if (md[0].barrel) { out[6] = cf.lhs[j]; out[7] = cf.rhs[j]; j++; }
    if (md[1].barrel) { out[8] = cf.lhs[j]; out[9] = cf.rhs[j]; j++; }
    out[10] = z0; out[11] = kO; out[12] = cf.n;
    return pass;
}

/* orc_eval_t3 out: [lhs/rhs T1, T2, T3], k */
int orc_eval_t3(const orc *o, const int32_t *mods3, const float *hits18, double *out)
{
    MDREC md[3];
    eval_mds(o, 3, mods3, hits18, md);
    CUTREC cf;
    float k;
    int pass = t3_cut_f(&o->K, &md[0], &md[1], &md[2], &cf, &k, NULL);
    for (int j = 0; j < 3; ++j) { out[2 * j] = cf.lhs[j]; out[2 * j + 1] = cf.rhs[j]; }
    out[6] = k;
    return pass;
}

/* the 40 scorer features of one triplet / quintuplet built from the given MDs */
int orc_eval_t3_features(const orc *o, const int32_t *mods3, const float *hits18, float *out40)
{
    MDREC md[3];
    eval_mds(o, 3, mods3, hits18, md);
    CUTREC cf;
    float k;
    T3AUX ax;
    int pass = t3_cut_f(&o->K, &md[0], &md[1], &md[2], &cf, &k, &ax);
    const MDREC *P[3] = {&md[0], &md[1], &md[2]};
    t3_features_f(&o->K, P, &ax, out40);
    return pass;
}

int orc_eval_t5_features(const orc *o, const int32_t *mods5, const float *hits30, float *out40)
{
    MDREC md[5];
    eval_mds(o, 5, mods5, hits30, md);
    CUTREC c3, cf;
    float kin, kout;
    t3_cut_f(&o->K, &md[0], &md[1], &md[2], &c3, &kin, NULL);
    t3_cut_f(&o->K, &md[2], &md[3], &md[4], &c3, &kout, NULL);
    const MDREC *P[5] = {&md[0], &md[1], &md[2], &md[3], &md[4]};
    T5AUX ax;
    int pass = t5_cut_f(&o->K, P, kin, kout, &cf, &ax);
    t5_features_f(&o->K, P, kin, kout, &ax, out40);
    return pass;
}

/* orc_eval_t5 out: [lhs/rhs Q1a, Q1b, Q2, Q3, Q4], kin, kout, kbr, resb, resd,
 * chi2_rphi, chi2_rz, score */
int orc_eval_t5(const orc *o, const int32_t *mods5, const float *hits30, double *out)
{
    MDREC md[5];
    eval_mds(o, 5, mods5, hits30, md);
    CUTREC c3;
    float kin, kout;
    t3_cut_f(&o->K, &md[0], &md[1], &md[2], &c3, &kin, NULL);
    t3_cut_f(&o->K, &md[2], &md[3], &md[4], &c3, &kout, NULL);
    const MDREC *P[5] = {&md[0], &md[1], &md[2], &md[3], &md[4]};
    CUTREC cf;
    T5AUX ax;
    int pass = t5_cut_f(&o->K, P, kin, kout, &cf, &ax);
    for (int j = 0; j < 5; ++j) { out[2 * j] = cf.lhs[j]; out[2 * j + 1] = cf.rhs[j]; }
    out[10] = kin; out[11] = kout; out[12] = ax.kbr; out[13] = ax.resb; out[14] = ax.resd;
    out[15] = ax.chi2p; out[16] = ax.chi2z; out[17] = ax.score;
    return pass;
}

/* FP64 margin (cut_margin) of one candidate of kind ORC_MD..ORC_T5 built from
 * the given MDs, as the chain would record it: the FP32 decision picks which
 * cuts can flip the outcome, the FP64 re-evaluation measures their relative
 * distance to threshold (infinite when two or more cuts fail).  For ORC_MD,
 * mods has one entry and hits six floats (lower, upper hit). */
double orc_eval_margin(const orc *o, int kind, const int32_t *mods, const float *hits)
{
    CUTREC cf, cd;
    if (kind == ORC_MD) {
        MDREC md;
        make_md(o, mods[0], &hits[0], &hits[3], &md, &cf, &cd);
        return cut_margin(&cf, &cd);
    }
    MDREC md[5];
    if (kind == ORC_SEG) {
        eval_mds(o, 2, mods, hits, md);
        float z0f, kOf;
        double z0d, kOd;
        seg_cut_f(&o->K, &md[0], &md[1], &cf, &z0f, &kOf);
        seg_cut_d(&o->K, &md[0], &md[1], &cd, &z0d, &kOd);
        return cut_margin(&cf, &cd);
    }
    if (kind == ORC_T3) {
        eval_mds(o, 3, mods, hits, md);
        float kf;
        double kd;
        t3_cut_f(&o->K, &md[0], &md[1], &md[2], &cf, &kf, NULL);
        t3_cut_d(&o->K, &md[0], &md[1], &md[2], &cd, &kd, NULL);
        return cut_margin(&cf, &cd);
    }
    if (kind == ORC_T5) {
        eval_mds(o, 5, mods, hits, md);
        CUTREC c3;
        float kin, kout;
        t3_cut_f(&o->K, &md[0], &md[1], &md[2], &c3, &kin, NULL);
        t3_cut_f(&o->K, &md[2], &md[3], &md[4], &c3, &kout, NULL);
        const MDREC *P[5] = {&md[0], &md[1], &md[2], &md[3], &md[4]};
        T5AUX af, ad;
        t5_cut_f(&o->K, P, kin, kout, &cf, &af);
        t5_cut_d(&o->K, P, kin, kout, &cd, &ad);
        return cut_margin(&cf, &cd);
    }
    return NAN;
}

/* ========================================================================= */
/* Pixel objects (Sec. 2.1 and the kernel-flow figure of Sec. 3): pixel line
 * segments (pLS, seeds of four pixel hits) linked to quintuplets (pT5) and
 * to triplets (pT3), cross-cleaning, track candidates (TC).  Runs on the
 * objects of the last orc_run.  The steps, in the paper's order:
 *   1. pT5: every (pLS, kept quintuplet) pair inside the linking window whose
 *      nine points pass the link chi2 cuts; within the collection a candidate
 *      survives iff no candidate sharing one of its hits (pixel or outer) has
 *      a smaller (score, seed, hit tuple) key;
 *   2. pT3: the same for pLS not used by a surviving pT5, with every triplet;
 *   3. pT3 near a surviving pT5 in eta-phi, or sharing a hit with one, are
 *      duplicates;
 *   4. kept quintuplets near a surviving pT5 or cleaned pT3, or sharing a hit
 *      with one, are duplicates;
 *   5. pLS used by neither are cleaned against all of the above (near, or
 *      sharing a pixel hit); among the rest a pLS sharing a pixel hit with a
 *      remaining pLS of smaller index is a duplicate;
 *   6. TC = surviving pT5, cleaned pT3, cleaned T5, cleaned pLS. */

static void pix_dir(const float *x, const float *y, const float *z, const int32_t *sd,
                    float *tx, float *ty, float *c)
{
    float x1 = x[sd[0]], y1 = y[sd[0]], z1 = z[sd[0]];
    float x4 = x[sd[3]], y4 = y[sd[3]], z4 = z[sd[3]];
    dir2_f(x1, y1, x4, y4, tx, ty);
    float dx = x4 - x1, dy = y4 - y1;
    *c = (z4 - z1) / sqrtf((dx * dx) + (dy * dy));
}

/* direction of an outer object from its first and last anchors A, E and its
 * curvature k: polar slope = dz / arc length */
static void obj_dir(const MDREC *A, const MDREC *E, float k, float *tx, float *ty, float *c)
{
    dir2_f(A->x, A->y, E->x, E->y, tx, ty);
    float dx = E->x - A->x, dy = E->y - A->y;
    *c = (E->z - A->z) / arc_f(sqrtf((dx * dx) + (dy * dy)), k);
}

/* bridge curvature of a quintuplet (its first, middle and last anchors) */
static float t5_kbr(const MDREC *A, const MDREC *C, const MDREC *E)
{
    float xac = C->x - A->x, yac = C->y - A->y;
    float xce = E->x - C->x, yce = E->y - C->y;
    float xae = E->x - A->x, yae = E->y - A->y;
    float lac = sqrtf((xac * xac) + (yac * yac));
    float lce = sqrtf((xce * xce) + (yce * yce));
    float lae = sqrtf((xae * xae) + (yae * yae));
    float crs = (xac * yae) - (yac * xae);
    return (2.0f * crs) / ((lac * lce) * lae);
}

static void lpt_md(const MDREC *m, lpt_f *p, lpt_d *q)
{
    p->x = m->x; p->y = m->y; p->z = m->z; p->sv = m->sv; p->r = m->r;
    p->kind = m->barrel ? 1 : 2;
    q->x = m->x; q->y = m->y; q->z = m->z; q->sv = m->sv; q->r = m->r; q->kind = p->kind;
}

static void lpt_px(float x, float y, float z, lpt_f *p, lpt_d *q)
{
    p->x = x; p->y = y; p->z = z; p->sv = 0.0f; p->r = 0.0f; p->kind = 0;
    q->x = x; q->y = y; q->z = z; q->sv = 0.0; q->r = 0.0; q->kind = 0;
}

/* hits of a candidate, as (kind, id): 4 pixel hits (kind 0), then the outer
 * hits of its object (kind 1) */
typedef struct { int n; int32_t id[14]; uint8_t kind[14]; } HITSET;

/* key order: score, then seed, then the outer hit tuple */
static int px_less(const PXREC *a, const int32_t *ta, const PXREC *b, const int32_t *tb, int w)
{
    if (a->score != b->score) return a->score < b->score;
    if (a->seed != b->seed) return a->seed < b->seed;
    for (int k = 0; k < w; ++k)
        if (ta[k] != tb[k]) return ta[k] < tb[k];
    return 0;
}

static int hits_share(const HITSET *a, const HITSET *b)
{
    for (int i = 0; i < a->n; ++i)
        for (int j = 0; j < b->n; ++j)
            if (a->kind[i] == b->kind[j] && a->id[i] == b->id[j]) return 1;
    return 0;
}

static void px_hits(const orc *o, const int32_t *seeds, const PXREC *c, int w, HITSET *h,
                    int32_t *tup)
{
    h->n = 0;
    for (int k = 0; k < 4; ++k) { h->id[h->n] = seeds[4 * c->seed + k]; h->kind[h->n++] = 0; }
    if (w == 10) {
        const T5REC *T = &((const T5REC *)o->t5.v)[c->obj];
        for (int j = 0; j < 5; ++j) md_hits(o, T->md[j], &tup[2 * j]);
    } else {
        const T3REC *T = &((const T3REC *)o->t3.v)[c->obj];
        md_hits(o, T->a, &tup[0]); md_hits(o, T->b, &tup[2]); md_hits(o, T->c, &tup[4]);
    }
    for (int k = 0; k < w; ++k) { h->id[h->n] = tup[k]; h->kind[h->n++] = 1; }
}

/* within a collection: keep[i] iff no candidate sharing a hit has a smaller
 * key (all pairs; collections are small) */
static void px_dedup(const orc *o, const int32_t *seeds, const gvec *v, int w, uint8_t *keep)
{
    const PXREC *C = (const PXREC *)v->v;
    int64_t n = v->n;
    HITSET *H = (HITSET *)malloc((size_t)(n > 0 ? n : 1) * sizeof(HITSET));
    int32_t *T = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * 10 * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) px_hits(o, seeds, &C[i], w, &H[i], &T[10 * i]);
    for (int64_t i = 0; i < n; ++i) {
        keep[i] = 1;
        for (int64_t j = 0; j < n && keep[i]; ++j)
            if (j != i && hits_share(&H[i], &H[j]) &&
                px_less(&C[j], &T[10 * j], &C[i], &T[10 * i], w))
                keep[i] = 0;
    }
    free(H); free(T);
}

int orc_run_pixel(orc *o, const double *pp, int n_pp, int32_t n_px, const float *x,
                  const float *y, const float *z, int32_t n_seeds, const int32_t *seeds)
{
    if (!o->keep || n_pp < ORC_PX_N_PARAMS || n_px < 0 || n_seeds < 0) return -1;
    for (int64_t i = 0; i < 4 * (int64_t)n_seeds; ++i)
        if (seeds[i] < 0 || seeds[i] >= n_px) return -1;
    gv_clear(&o->pt5); gv_clear(&o->pt3); gv_clear(&o->tc);
    free(o->pt5_keep); free(o->pt3_keep); free(o->t5_clean); free(o->pls_keep); free(o->seeds);
    o->n_seeds = n_seeds; o->n_px = n_px; o->px_near = 0;
    o->seeds = (int32_t *)malloc((size_t)(n_seeds > 0 ? n_seeds : 1) * 4 * sizeof(int32_t));
    memcpy(o->seeds, seeds, (size_t)n_seeds * 4 * sizeof(int32_t));
    const KCONST *K = &o->K;
    /* pixel constants, each rounded once to FP32 */
    const float sig2p = (float)(pp[ORC_PX_SIGRPHI] * pp[ORC_PX_SIGRPHI]);
    const float sigz = (float)pp[ORC_PX_SIGZ];
    const double wl = pp[ORC_PX_WLINK] * (double)K->w;
    const float wl2 = (float)(wl * wl);
    const float dr2 = (float)pp[ORC_PX_DR2];
    const float x5p = (float)pp[ORC_PX_X5P], x5z = (float)pp[ORC_PX_X5Z];
    const float x3p = (float)pp[ORC_PX_X3P], x3z = (float)pp[ORC_PX_X3Z];
    const MDREC *MD = (const MDREC *)o->md.v;
    const T3REC *T3 = (const T3REC *)o->t3.v;
    const T5REC *T5 = (const T5REC *)o->t5.v;
    const int64_t n3 = o->t3.n, n5 = o->t5.n;

    /* directions: pLS from its first and last pixel hits, outer objects from
     * their first and last anchors */
    float *sd = (float *)malloc((size_t)(n_seeds > 0 ? n_seeds : 1) * 3 * sizeof(float));
    for (int32_t i = 0; i < n_seeds; ++i)
        pix_dir(x, y, z, &seeds[4 * i], &sd[3 * i], &sd[3 * i + 1], &sd[3 * i + 2]);
    float *d5 = (float *)malloc((size_t)(n5 > 0 ? n5 : 1) * 3 * sizeof(float));
    for (int64_t t = 0; t < n5; ++t) {
        const MDREC *A = &MD[T5[t].md[0]], *C = &MD[T5[t].md[2]], *E = &MD[T5[t].md[4]];
        obj_dir(A, E, t5_kbr(A, C, E), &d5[3 * t], &d5[3 * t + 1], &d5[3 * t + 2]);
    }
    float *d3 = (float *)malloc((size_t)(n3 > 0 ? n3 : 1) * 3 * sizeof(float));
    for (int64_t t = 0; t < n3; ++t)
        obj_dir(&MD[T3[t].a], &MD[T3[t].c], T3[t].k, &d3[3 * t], &d3[3 * t + 1], &d3[3 * t + 2]);

    /* 1. pT5 */
    for (int32_t i = 0; i < n_seeds; ++i) {
        const int32_t *h = &seeds[4 * i];
        for (int64_t t = 0; t < n5; ++t) {
            if (!o->keep[t]) continue;
            CUTREC wf, wd;
            int pw = link_window_f(sd[3 * i], sd[3 * i + 1], sd[3 * i + 2], d5[3 * t],
                                   d5[3 * t + 1], d5[3 * t + 2], wl2, &wf);
            link_window_d(sd[3 * i], sd[3 * i + 1], sd[3 * i + 2], d5[3 * t], d5[3 * t + 1],
                          d5[3 * t + 2], wl2, &wd);
            if (cut_margin(&wf, &wd) < NEAR_REL) o->px_near++;
            if (!pw) continue;
            lpt_f pf[9]; lpt_d pd[9];
            for (int k = 0; k < 4; ++k) lpt_px(x[h[k]], y[h[k]], z[h[k]], &pf[k], &pd[k]);
            for (int j = 0; j < 5; ++j) lpt_md(&MD[T5[t].md[j]], &pf[4 + j], &pd[4 + j]);
            CUTREC cf, cd;
            float sc;
            double scd;
            int pass = link_cut_f(K, pf, 9, 6, sig2p, sigz, x5p, x5z, &cf, &sc);
            link_cut_d(K, pd, 9, 6, sig2p, sigz, x5p, x5z, &cd, &scd);
            if (cut_margin(&cf, &cd) < NEAR_REL) o->px_near++;
            if (pass) {
                PXREC *r = (PXREC *)gv_push(&o->pt5);
                r->seed = i; r->obj = (int32_t)t; r->score = sc;
            }
        }
    }
    o->pt5_keep = (uint8_t *)malloc((size_t)(o->pt5.n > 0 ? o->pt5.n : 1));
    px_dedup(o, seeds, &o->pt5, 10, o->pt5_keep);
    uint8_t *used = (uint8_t *)calloc((size_t)(n_seeds > 0 ? n_seeds : 1), 1);
    const PXREC *P5 = (const PXREC *)o->pt5.v;
    for (int64_t c = 0; c < o->pt5.n; ++c)
        if (o->pt5_keep[c]) used[P5[c].seed] = 1;

    /* 2. pT3 from the unused pLS */
    for (int32_t i = 0; i < n_seeds; ++i) {
        if (used[i]) continue;
        const int32_t *h = &seeds[4 * i];
        for (int64_t t = 0; t < n3; ++t) {
            CUTREC wf, wd;
            int pw = link_window_f(sd[3 * i], sd[3 * i + 1], sd[3 * i + 2], d3[3 * t],
                                   d3[3 * t + 1], d3[3 * t + 2], wl2, &wf);
            link_window_d(sd[3 * i], sd[3 * i + 1], sd[3 * i + 2], d3[3 * t], d3[3 * t + 1],
                          d3[3 * t + 2], wl2, &wd);
            if (cut_margin(&wf, &wd) < NEAR_REL) o->px_near++;
            if (!pw) continue;
            lpt_f pf[7]; lpt_d pd[7];
            for (int k = 0; k < 4; ++k) lpt_px(x[h[k]], y[h[k]], z[h[k]], &pf[k], &pd[k]);
            lpt_md(&MD[T3[t].a], &pf[4], &pd[4]);
            lpt_md(&MD[T3[t].b], &pf[5], &pd[5]);
            lpt_md(&MD[T3[t].c], &pf[6], &pd[6]);
            CUTREC cf, cd;
            float sc;
            double scd;
            int pass = link_cut_f(K, pf, 7, 4, sig2p, sigz, x3p, x3z, &cf, &sc);
            link_cut_d(K, pd, 7, 4, sig2p, sigz, x3p, x3z, &cd, &scd);
            if (cut_margin(&cf, &cd) < NEAR_REL) o->px_near++;
            if (pass) {
                PXREC *r = (PXREC *)gv_push(&o->pt3);
                r->seed = i; r->obj = (int32_t)t; r->score = sc;
            }
        }
    }
    o->pt3_keep = (uint8_t *)malloc((size_t)(o->pt3.n > 0 ? o->pt3.n : 1));
    px_dedup(o, seeds, &o->pt3, 6, o->pt3_keep);
    const PXREC *P3 = (const PXREC *)o->pt3.v;

    /* hit sets of the surviving pT5 */
    HITSET hs;
    int32_t tup[10];
    int64_t np5 = o->pt5.n, np3 = o->pt3.n;

    /* 3. pT3 against the surviving pT5 */
    for (int64_t c = 0; c < np3; ++c) {
        if (!o->pt3_keep[c]) continue;
        HITSET hc;
        int32_t tc[10];
        px_hits(o, seeds, &P3[c], 6, &hc, tc);
        const float *a = &sd[3 * P3[c].seed];
        for (int64_t u = 0; u < np5 && o->pt3_keep[c]; ++u) {
            if (!o->pt5_keep[u]) continue;
            px_hits(o, seeds, &P5[u], 10, &hs, tup);
            const float *b = &sd[3 * P5[u].seed];
            CUTREC ff, fd;
            int near = close_cut_f(a[0], a[1], a[2], b[0], b[1], b[2], dr2, &ff);
            close_cut_d(a[0], a[1], a[2], b[0], b[1], b[2], dr2, &fd);
            if (cut_margin(&ff, &fd) < NEAR_REL) o->px_near++;
            if (near || hits_share(&hc, &hs)) o->pt3_keep[c] = 0;
        }
    }

    /* 4. kept quintuplets against the surviving pT5 and cleaned pT3 */
    o->t5_clean = (uint8_t *)malloc((size_t)(n5 > 0 ? n5 : 1));
    for (int64_t t = 0; t < n5; ++t) {
        o->t5_clean[t] = o->keep[t];
        if (!o->keep[t]) continue;
        HITSET ht;
        ht.n = 0;
        for (int j = 0; j < 5; ++j) {
            md_hits(o, T5[t].md[j], &tup[2 * j]);
        }
        for (int k = 0; k < 10; ++k) { ht.id[ht.n] = tup[k]; ht.kind[ht.n++] = 1; }
        const float *a = &d5[3 * t];
        for (int pass = 0; pass < 2 && o->t5_clean[t]; ++pass) {
            const gvec *v = pass ? &o->pt3 : &o->pt5;
            const uint8_t *kp = pass ? o->pt3_keep : o->pt5_keep;
            const PXREC *Q = (const PXREC *)v->v;
            for (int64_t u = 0; u < v->n && o->t5_clean[t]; ++u) {
                if (!kp[u]) continue;
                int32_t tu[10];
                px_hits(o, seeds, &Q[u], pass ? 6 : 10, &hs, tu);
                const float *b = &sd[3 * Q[u].seed];
                CUTREC ff, fd;
                int near = close_cut_f(a[0], a[1], a[2], b[0], b[1], b[2], dr2, &ff);
                close_cut_d(a[0], a[1], a[2], b[0], b[1], b[2], dr2, &fd);
                if (cut_margin(&ff, &fd) < NEAR_REL) o->px_near++;
                if (near || hits_share(&ht, &hs)) o->t5_clean[t] = 0;
            }
        }
    }

    /* 5. pLS used by neither, against everything above, then among themselves */
    for (int64_t c = 0; c < np3; ++c)
        if (o->pt3_keep[c]) used[P3[c].seed] = 1;
    o->pls_keep = (uint8_t *)malloc((size_t)(n_seeds > 0 ? n_seeds : 1));
    for (int32_t i = 0; i < n_seeds; ++i) {
        o->pls_keep[i] = !used[i];
        if (used[i]) continue;
        HITSET hi;
        hi.n = 4;
        for (int k = 0; k < 4; ++k) { hi.id[k] = seeds[4 * i + k]; hi.kind[k] = 0; }
        const float *a = &sd[3 * i];
        for (int pass = 0; pass < 3 && o->pls_keep[i]; ++pass) {
            int64_t n = pass == 0 ? np5 : pass == 1 ? np3 : n5;
            for (int64_t u = 0; u < n && o->pls_keep[i]; ++u) {
                const float *b;
                int share = 0;
                if (pass < 2) {
                    const PXREC *Q = pass ? &P3[u] : &P5[u];
                    if (!(pass ? o->pt3_keep[u] : o->pt5_keep[u])) continue;
                    HITSET hq;
                    hq.n = 4;
                    for (int k = 0; k < 4; ++k) { hq.id[k] = seeds[4 * Q->seed + k]; hq.kind[k] = 0; }
                    share = hits_share(&hi, &hq);
                    b = &sd[3 * Q->seed];
                } else {
                    if (!o->t5_clean[u]) continue;
                    b = &d5[3 * u];
                }
                CUTREC ff, fd;
                int near = close_cut_f(a[0], a[1], a[2], b[0], b[1], b[2], dr2, &ff);
                close_cut_d(a[0], a[1], a[2], b[0], b[1], b[2], dr2, &fd);
                if (cut_margin(&ff, &fd) < NEAR_REL) o->px_near++;
                if (near || share) o->pls_keep[i] = 0;
            }
        }
    }
    /* among the remaining pLS: a smaller index sharing a pixel hit wins */
    uint8_t *rem = (uint8_t *)malloc((size_t)(n_seeds > 0 ? n_seeds : 1));
    memcpy(rem, o->pls_keep, (size_t)(n_seeds > 0 ? n_seeds : 1));
    for (int32_t i = 0; i < n_seeds; ++i) {
        if (!rem[i]) continue;
        for (int32_t j = 0; j < i && o->pls_keep[i]; ++j) {
            if (!rem[j]) continue;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    if (seeds[4 * i + a] == seeds[4 * j + b]) o->pls_keep[i] = 0;
        }
    }
    free(rem);

    /* 6. track candidates */
    for (int64_t c = 0; c < np5; ++c) {
        if (!o->pt5_keep[c]) continue;
        TCREC *r = (TCREC *)gv_push(&o->tc);
        r->type = ORC_TC_PT5; r->seed = P5[c].seed;
        for (int j = 0; j < 5; ++j) md_hits(o, T5[P5[c].obj].md[j], &r->hits[2 * j]);
    }
    for (int64_t c = 0; c < np3; ++c) {
        if (!o->pt3_keep[c]) continue;
        TCREC *r = (TCREC *)gv_push(&o->tc);
        r->type = ORC_TC_PT3; r->seed = P3[c].seed;
        const T3REC *T = &T3[P3[c].obj];
        md_hits(o, T->a, &r->hits[0]); md_hits(o, T->b, &r->hits[2]); md_hits(o, T->c, &r->hits[4]);
        for (int k = 6; k < 10; ++k) r->hits[k] = -1;
    }
    for (int64_t t = 0; t < n5; ++t) {
        if (!o->t5_clean[t]) continue;
        TCREC *r = (TCREC *)gv_push(&o->tc);
        r->type = ORC_TC_T5; r->seed = -1;
        for (int j = 0; j < 5; ++j) md_hits(o, T5[t].md[j], &r->hits[2 * j]);
    }
    for (int32_t i = 0; i < n_seeds; ++i) {
        if (!o->pls_keep[i]) continue;
        TCREC *r = (TCREC *)gv_push(&o->tc);
        r->type = ORC_TC_PLS; r->seed = i;
        for (int k = 0; k < 10; ++k) r->hits[k] = -1;
    }
    free(used); free(sd); free(d5); free(d3);
    return 0;
}

int64_t orc_px_count(const orc *o, int what)
{
    int64_t c = 0;
    switch (what) {
    case 0: return o->pt5.n;
    case 1: for (int64_t i = 0; i < o->pt5.n; ++i) c += o->pt5_keep[i]; return c;
    case 2: return o->pt3.n;
    case 3: for (int64_t i = 0; i < o->pt3.n; ++i) c += o->pt3_keep[i]; return c;
    case 4: return o->tc.n;
    case 5: return o->px_near;
    }
    return -1;
}

/* candidates of pT5 (what 0) or pT3 (what 2): seed, object tuple (10 or 6
 * hits, -1 padded), score bits, survived the collection's dedup */
void orc_px_candidates(const orc *o, int what, int32_t *out13)
{
    const gvec *v = what == 0 ? &o->pt5 : &o->pt3;
    const PXREC *C = (const PXREC *)v->v;
    const uint8_t *kp = what == 0 ? o->pt5_keep : o->pt3_keep;
    for (int64_t i = 0; i < v->n; ++i) {
        int32_t *r = &out13[13 * i];
        HITSET h;
        int32_t tup[10];
        for (int k = 0; k < 10; ++k) tup[k] = -1;
        px_hits(o, o->seeds, &C[i], what == 0 ? 10 : 6, &h, tup);
        r[0] = C[i].seed;
        memcpy(&r[1], tup, sizeof(tup));
        memcpy(&r[11], &C[i].score, sizeof(float));
        r[12] = kp[i];
    }
}

void orc_tc(const orc *o, int32_t *out12)
{
    const TCREC *T = (const TCREC *)o->tc.v;
    for (int64_t i = 0; i < o->tc.n; ++i) {
        out12[12 * i] = T[i].type;
        out12[12 * i + 1] = T[i].seed;
        memcpy(&out12[12 * i + 2], T[i].hits, sizeof(T[i].hits));
    }
}

/* Single-candidate evaluation of a pixel link (closed-form checks): a pLS of
 * four pixel hits (pix12: x, y, z of each, inner to outer) with the outer
 * object built from n_md = 5 (quintuplet) or 3 (triplet) MDs given as
 * (module, lower hit, upper hit).  out: pLS tx, ty, cot; object tx, ty, cot;
 * window dot, sin^2, polar term; chi2_rphi, chi2_rz, score.  Returns the
 * FP32 decision of window and chi2 cuts together. */
int orc_eval_link(const orc *o, const double *pp, const float *pix12, int n_md,
                  const int32_t *mods, const float *hits, double *out)
{
    if (n_md != 3 && n_md != 5) return -1;
    MDREC md[5];
    eval_mds(o, n_md, mods, hits, md);
    const KCONST *K = &o->K;
    float x[4], y[4], z[4];
    for (int k = 0; k < 4; ++k) { x[k] = pix12[3 * k]; y[k] = pix12[3 * k + 1]; z[k] = pix12[3 * k + 2]; }
    const int32_t sd[4] = {0, 1, 2, 3};
    float ptx, pty, pc, otx, oty, oc;
    pix_dir(x, y, z, sd, &ptx, &pty, &pc);
    float k = 0.0f;
    if (n_md == 5) {
        k = t5_kbr(&md[0], &md[2], &md[4]);
    } else {
        CUTREC c3;
        t3_cut_f(K, &md[0], &md[1], &md[2], &c3, &k, NULL);
    }
    obj_dir(&md[0], &md[n_md - 1], k, &otx, &oty, &oc);
    const double wl = pp[ORC_PX_WLINK] * (double)K->w;
    CUTREC wf;
    int pw = link_window_f(ptx, pty, pc, otx, oty, oc, (float)(wl * wl), &wf);
    lpt_f pf[9]; lpt_d pd[9];
    for (int j = 0; j < 4; ++j) lpt_px(x[j], y[j], z[j], &pf[j], &pd[j]);
    for (int j = 0; j < n_md; ++j) lpt_md(&md[j], &pf[4 + j], &pd[4 + j]);
    CUTREC cf;
    float sc;
    const float sig2p = (float)(pp[ORC_PX_SIGRPHI] * pp[ORC_PX_SIGRPHI]);
    int pass = n_md == 5
        ? link_cut_f(K, pf, 9, 6, sig2p, (float)pp[ORC_PX_SIGZ], (float)pp[ORC_PX_X5P],
                     (float)pp[ORC_PX_X5Z], &cf, &sc)
        : link_cut_f(K, pf, 7, 4, sig2p, (float)pp[ORC_PX_SIGZ], (float)pp[ORC_PX_X3P],
                     (float)pp[ORC_PX_X3Z], &cf, &sc);
    out[0] = ptx; out[1] = pty; out[2] = pc; out[3] = otx; out[4] = oty; out[5] = oc;
    out[6] = -wf.lhs[0]; out[7] = wf.lhs[1]; out[8] = wf.lhs[2];
    out[9] = cf.lhs[0]; out[10] = cf.lhs[1]; out[11] = sc;
    return pw && pass;
}
