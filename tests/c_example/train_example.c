/*
 * A plain C consumer of the library: no Python, no torch.  It builds a small
 * seeded training set on the host (windows of 16x16; positives carry a dark
 * horizontal band, negatives are noise), copies it to HIP device memory,
 * trains a few rounds through the C ABI and checks the records.
 *
 * Usage: train_example [n_windows] [rounds]   (defaults 600 and 5)
 * Prints one line per round; exits 0 when every check holds.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "vjboost.h"

static uint32_t lcg(uint32_t *s) { *s = *s * 1664525u + 1013904223u; return *s >> 8; }

static int fail(const char *what) {
    fprintf(stderr, "FAIL: %s: %s\n", what, boost_last_error());
    return 1;
}

int main(int argc, char **argv) {
    const int64_t n = argc > 1 ? atoll(argv[1]) : 600;
    const int32_t rounds = argc > 2 ? atoi(argv[2]) : 5;
    const int W = 16, H = 16;
    if (n < 2 || rounds < 1) { fprintf(stderr, "bad arguments\n"); return 2; }
    uint8_t *img = (uint8_t *)malloc((size_t)n * W * H), *lab = (uint8_t *)malloc((size_t)n);
    boost_stump *rec = (boost_stump *)malloc(sizeof(boost_stump) * (size_t)rounds);
    if (!img || !lab || !rec) return 2;
    uint32_t seed = 12345u;
    for (int64_t i = 0; i < n; ++i) {
        lab[i] = (uint8_t)(i % 3 == 0);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int v = 96 + (int)(lcg(&seed) % 64);
                if (lab[i] && y >= 5 && y < 8) v -= 60;
                img[(i * H + y) * W + x] = (uint8_t)v;
            }
    }
    boost_feature_set fs = {W, H, 0x1F};
    boost_options o;
    if (boost_options_default(&o) != BOOST_OK) return fail("options");
    const int64_t F = boost_feature_count(&fs);
    const size_t ws = boost_workspace_bytes(n, &fs, &o);
    if (F <= 0 || ws == 0) return fail("sizes");
    void *d_img = NULL, *d_lab = NULL, *d_ws = NULL;
    if (hipMalloc(&d_img, (size_t)n * W * H) != hipSuccess || hipMalloc(&d_lab, (size_t)n) != hipSuccess ||
        hipMalloc(&d_ws, ws) != hipSuccess) {
        fprintf(stderr, "FAIL: hipMalloc\n");
        return 1;
    }
    if (hipMemcpy(d_img, img, (size_t)n * W * H, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_lab, lab, (size_t)n, hipMemcpyHostToDevice) != hipSuccess) {
        fprintf(stderr, "FAIL: hipMemcpy\n");
        return 1;
    }
    boost_ctx *ctx = NULL;
    if (boost_init(&ctx, (const uint8_t *)d_img, (const uint8_t *)d_lab, n, &fs, &o, d_ws, ws) != BOOST_OK)
        return fail("boost_init");
    /* the inputs may be freed once boost_init returns */
    hipFree(d_img);
    hipFree(d_lab);
    if (boost_train(ctx, rounds, rec) != BOOST_OK) return fail("boost_train");
    int bad = 0;
    for (int32_t t = 0; t < rounds; ++t) {
        const boost_stump *s = &rec[t];
        boost_feature f;
        if (boost_feature_desc(&fs, s->feature, &f) != BOOST_OK) return fail("boost_feature_desc");
        printf("round %d feature %lld type %d at (%d,%d) cell %dx%d polarity %d threshold %d error %.9g alpha %.6g\n",
               s->round, (long long)s->feature, f.type, f.x, f.y, f.cell_w, f.cell_h, s->polarity, s->threshold,
               s->error_raw, s->alpha);
        bad |= s->round != t || s->feature < 0 || s->feature >= F || f.type != s->type || f.x != s->x ||
               (s->polarity != 1 && s->polarity != -1) || !(s->error_raw >= 0.0 && s->error_raw < 0.5) ||
               !(s->alpha > 0.0);
    }
    int32_t done = -1;
    if (boost_rounds_done(ctx, &done) != BOOST_OK || done != rounds) bad = 1;
    /* the first stump separates the band from the noise */
    bad |= !(rec[0].error_raw < 0.05);
    boost_destroy(ctx);
    hipFree(d_ws);
    free(img); free(lab); free(rec);
    if (bad) { fprintf(stderr, "FAIL: record checks\n"); return 1; }
    printf("ok: %d rounds over %lld windows and %lld features\n", rounds, (long long)n, (long long)F);
    return 0;
}
