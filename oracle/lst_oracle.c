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

/* ------------------------------------------------------------------------- */
typedef struct {
    float kmax, klim, kh, tolu, tolv, tolkc, epsak;
    float z0max, sigu, sigv, nsig, d0max, w, w2, xrphi, xrz;
} KCONST;

typedef struct {
    float cx, cy, cz, ux, uy, uz, vx, vy, vz, g, rl;
    int barrel;
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


int orc_run(orc *o, int32_t n_hits, const float *x, const float *y, const float *z,
            const int32_t *module, const uint8_t *sensor)
{
    if (n_hits < 0) return -1;
    for (int32_t h = 0; h < n_hits; ++h)
        if (module[h] < 0 || module[h] >= o->n_mod || sensor[h] > 1) return -1;
    free_event(o);
    gv_clear(&o->md); gv_clear(&o->seg); gv_clear(&o->t3); gv_clear(&o->t5);
    for (int k = 0; k < 4; ++k) gv_clear(&o->near[k]);
    memset(o->cand, 0, sizeof(o->cand));
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
                int pass = make_md(o, m, L, U, &md, &cf, &cd);
                md.hlo = hl; md.hup = hu;
                double mg = cut_margin(&cf, &cd);
                if (pass) *(MDREC *)gv_push(&o->md) = md;
                if (mg < NEAR_REL) {
                    NEARREC *r = (NEARREC *)gv_push(&o->near[0]);
                    memset(r->hits, 0xff, sizeof(r->hits));
                    r->hits[0] = hl; r->hits[1] = hu;
                    r->margin = mg; r->decision = (uint8_t)pass;
                }
            }
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
                    seg_cut_d(&o->K, &MD[i], &MD[j], &cd, &z0d, &kOd);
                    if (pass) {
                        SEGREC *s = (SEGREC *)gv_push(&o->seg);
                        s->i = i; s->o = j;
                    }
                    double mg = cut_margin(&cf, &cd);
                    if (mg < NEAR_REL) {
                        int32_t mds[2] = {i, j};
                        push_near(o, 1, mds, 2, mg, pass);
                    }
                }
            }
        }
    }
    o->seg_off[n_md] = (int32_t)o->seg.n;
    free(md_off);
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
                    t3_cut_d(&o->K, &MD[a], &MD[b], &MD[c], &cd, &kd, NULL);
                    if (pass) {
                        T3REC *t = (T3REC *)gv_push(&o->t3);
                        t->a = (int32_t)a; t->b = b; t->c = c; t->k = kf;
                        const MDREC *P3[3] = {&MD[a], &MD[b], &MD[c]};
                        t3_features_f(&o->K, P3, &ax, t->feat);
                    }
                    double mg = cut_margin(&cf, &cd);
                    if (mg < NEAR_REL) {
                        int32_t mds[3] = {(int32_t)a, b, c};
                        push_near(o, 2, mds, 3, mg, pass);
                    }
                }
            }
        }
        o->t3_off[n_md] = (int32_t)o->t3.n;
    }
    o->n_hits = n_hits;
    run_t5_dedup(o);
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
            t5_cut_d(&o->K, P, T3[t].k, T3[t2].k, &cd, &ad);
            int32_t mds[5] = {T3[t].a, T3[t].b, c, T3[t2].b, T3[t2].c};
            if (pass) {
                T5REC *q = (T5REC *)gv_push(&o->t5);
                memcpy(q->md, mds, sizeof(mds));
                q->score = (float)af.score;
                t5_features_f(&o->K, P, T3[t].k, T3[t2].k, &af, q->feat);
            }
            double mg = cut_margin(&cf, &cd);
            if (mg < NEAR_REL) push_near(o, 3, mds, 5, mg, pass);
        }
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
