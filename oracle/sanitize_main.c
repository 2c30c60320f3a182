/* Test driver of the oracle for sanitizer builds (TEST INFRASTRUCTURE).
 *
 * Reads one input file (written by tests/test_oracle_sanitizers.py):
 *   int32 n_params, n_mod, n_events; double params[n_params];
 *   float mod_f32[21 * n_mod]; int32 mod_i32[4 * n_mod];
 *   per event: int32 n_hits; float x[n], y[n], z[n]; int32 module[n]; uint8 sensor[n]
 * runs every event through the whole chain, reads every output array, reruns
 * the quintuplets with every seventh triplet vetoed, and prints per event
 *   n_md n_seg n_t3 n_t5 n_kept n_t5_rerun n_kept_rerun
 * so that the caller can compare with the oracle built without sanitizers.
 * Built and run only by that test, with -fsanitize=address,undefined.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "lst_oracle.h"

static void *xread(FILE *f, size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p || (n && fread(p, 1, n, f) != n)) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[3];
    if (fread(hdr, sizeof(int32_t), 3, f) != 3) return 2;
    const int np = hdr[0], nm = hdr[1], ne = hdr[2];
    double *params = xread(f, sizeof(double) * np);
    float *f32 = xread(f, sizeof(float) * 21 * (size_t)nm);
    int32_t *i32 = xread(f, sizeof(int32_t) * 4 * (size_t)nm);
    orc *o = orc_create(params, np, nm, f32, i32);
    if (!o) return 3;
    static const int width[5] = {2, 4, 6, 10, 10};
    for (int e = 0; e < ne; ++e) {
        int32_t n;
        if (fread(&n, sizeof(n), 1, f) != 1) return 2;
        float *x = xread(f, sizeof(float) * n), *y = xread(f, sizeof(float) * n),
              *z = xread(f, sizeof(float) * n);
        int32_t *mod = xread(f, sizeof(int32_t) * n);
        uint8_t *sen = xread(f, n);
        if (orc_run(o, n, x, y, z, mod, sen) != 0) return 4;
        int64_t cnt[5];
        for (int k = 0; k < 5; ++k) {
            cnt[k] = orc_count(o, k);
            int32_t *t = malloc(sizeof(int32_t) * width[k] * (size_t)(cnt[k] + 1));
            orc_tuples(o, k, t);
            free(t);
        }
        int64_t cands[4];
        orc_cands(o, cands);
        float *sc = malloc(sizeof(float) * (size_t)(cnt[3] + 1));
        uint8_t *kp = malloc((size_t)cnt[3] + 1);
        float *k3 = malloc(sizeof(float) * (size_t)(cnt[2] + 1));
        float *f5 = malloc(sizeof(float) * 40 * (size_t)(cnt[3] + 1));
        float *f3 = malloc(sizeof(float) * 40 * (size_t)(cnt[2] + 1));
        orc_t5_scores(o, sc);
        orc_t5_keep(o, kp);
        orc_t3_curv(o, k3);
        orc_t5_features(o, f5);
        orc_t3_features(o, f3);
        for (int k = 0; k < 4; ++k) {
            int64_t nn = orc_near_count(o, k);
            int32_t *tt = malloc(sizeof(int32_t) * width[k] * (size_t)(nn + 1));
            double *mg = malloc(sizeof(double) * (size_t)(nn + 1));
            uint8_t *dc = malloc((size_t)nn + 1);
            orc_near(o, k, tt, mg, dc);
            free(tt); free(mg); free(dc);
        }
        uint8_t *veto = calloc((size_t)cnt[2] + 1, 1);
        for (int64_t i = 0; i < cnt[2]; i += 7) veto[i] = 1;
        if (orc_rerun_t5(o, veto) != 0) return 5;
        printf("%lld %lld %lld %lld %lld %lld %lld\n", (long long)cnt[0], (long long)cnt[1],
               (long long)cnt[2], (long long)cnt[3], (long long)cnt[4],
               (long long)orc_count(o, 3), (long long)orc_count(o, 4));
        free(veto); free(sc); free(kp); free(k3); free(f5); free(f3);
        free(x); free(y); free(z); free(mod); free(sen);
    }
    orc_destroy(o);
    free(params); free(f32); free(i32);
    fclose(f);
    return 0;
}
