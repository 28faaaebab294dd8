/*
 * vj_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for Viola-Jones discrete AdaBoost training
 * (arXiv 1306.1467, Sections 2.1-2.3).  Only the tests, the package's smoke
 * check and the benchmark's CPU-baseline leg use it; the product path never
 * calls, links or loads it, and it shares no code with the HIP library.
 *
 * Every routine follows the paper's definitions directly:
 *   - integral image: Section 2.1, the equation for i(x, y);
 *   - rectangle sum from four integral-image corners: Section 2.1, Figure 2 text;
 *   - Haar features of five types, their enumeration and counts: Section 2.2;
 *   - the decision stump h(x, f, p, theta): Section 2.2, stump equation;
 *   - weights, normalisation, error, update, beta, alpha: Section 2.3 and the
 *     master/slave pseudocode of Section 3.3.2.
 * Readings where the paper is silent are stated where they are used.
 *
 * Conventions:
 *   window W x H, images row-major uint8 [N][H][W];
 *   integral image ii[(H+1)][(W+1)] int32 with a zero first row and column,
 *     ii[y][x] = sum of o(x', y') over x' < x, y' < y (the paper's inclusive
 *     i(x, y) shifted by one so that empty rectangles need no special case);
 *   feature descriptor int32[5] = {type, x, y, cw, ch};
 *   types: 0 = three-rect horizontal, 1 = three-rect vertical,
 *          2 = two-rect horizontal, 3 = two-rect vertical, 4 = four-rect
 *     (the order in which Section 2.2 adds the counts and in which Section
 *     3.3.2 assigns the feature groups to slaves).
 *
 * Parallelism: loops over independent features may use OpenMP; nothing inside
 * one feature is reordered, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Base cell counts (columns, rows) of each feature type, Section 2.2:
 * the smallest three-rectangle feature is 3x1 pixels, the smallest
 * two-rectangle feature 2x1, the four-rectangle one 2x2. */
static const int BASE_W[5] = {3, 1, 2, 1, 2};
static const int BASE_H[5] = {1, 3, 1, 2, 2};

/* ---------------------------------------------------------------- Section 2.2
 * Enumeration.  Reading (the paper gives only the counts): every feature is its
 * base shape with each cell scaled independently to cw x ch pixels, cw, ch >= 1,
 * placed at every position where it fits.  Global order: type, then cw, then
 * ch, then y, then x (x fastest).  This reproduces the printed 43,200 /
 * 27,600 / 20,736 per type and 162,336 in total for 24x24. */
int64_t or_feature_count(int W, int H, int type_mask)
{
    int64_t total = 0;
    for (int t = 0; t < 5; ++t) {
        if (!(type_mask & (1 << t))) continue;
        for (int cw = 1; BASE_W[t] * cw <= W; ++cw)
            for (int ch = 1; BASE_H[t] * ch <= H; ++ch)
                for (int y = 0; y + BASE_H[t] * ch <= H; ++y)
                    for (int x = 0; x + BASE_W[t] * cw <= W; ++x)
                        ++total;
    }
    return total;
}

int64_t or_enumerate(int W, int H, int type_mask, int32_t *out)
{
    int64_t j = 0;
    for (int t = 0; t < 5; ++t) {
        if (!(type_mask & (1 << t))) continue;
        for (int cw = 1; BASE_W[t] * cw <= W; ++cw)
            for (int ch = 1; BASE_H[t] * ch <= H; ++ch)
                for (int y = 0; y + BASE_H[t] * ch <= H; ++y)
                    for (int x = 0; x + BASE_W[t] * cw <= W; ++x) {
                        int32_t *d = out + 5 * j;
                        d[0] = t; d[1] = x; d[2] = y; d[3] = cw; d[4] = ch;
                        ++j;
                    }
    }
    return j;
}

/* ---------------------------------------------------------------- Section 2.1
 * Integral image: the sum of all pixels above and to the left. */
void or_integral(const uint8_t *img, int W, int H, int32_t *ii)
{
    const int S = W + 1;
    for (int x = 0; x <= W; ++x) ii[x] = 0;
    for (int y = 1; y <= H; ++y) {
        ii[y * S] = 0;
        for (int x = 1; x <= W; ++x) {
            int32_t s = 0;
            for (int yy = 0; yy < y; ++yy)
                for (int xx = 0; xx < x; ++xx)
                    s += img[yy * W + xx];
            ii[y * S + x] = s;
        }
    }
}

/* Rectangle sum with four corner look-ups, Section 2.1: with corners
 * 1 = top-left, 2 = top-right, 3 = bottom-left, 4 = bottom-right,
 * sum = 4 + 1 - (2 + 3). */
static int32_t rect_sum(const int32_t *ii, int W, int x, int y, int w, int h)
{
    const int S = W + 1;
    int32_t c1 = ii[y * S + x];
    int32_t c2 = ii[y * S + x + w];
    int32_t c3 = ii[(y + h) * S + x];
    int32_t c4 = ii[(y + h) * S + x + w];
    return c4 + c1 - (c2 + c3);
}

int32_t or_rect_sum(const int32_t *ii, int W, int x, int y, int w, int h)
{
    return rect_sum(ii, W, x, y, w, h);
}

/* Feature value, Section 2.2: the sum over the dark rectangles minus the sum
 * over the white ones.  Figure 3 (which shows the shading) is missing from the
 * text, so the shading is a reading:
 *   two-rect horizontal  [white | dark]             -> right - left
 *   two-rect vertical    [white / dark]             -> bottom - top
 *   three-rect horizontal [white | dark | white]    -> middle - left - right
 *   three-rect vertical   the same, stacked         -> middle - top - bottom
 *   four-rect [white dark / dark white]             -> TR + BL - TL - BR
 * Three-rect features are unweighted, as the text states a plain difference. */
int32_t or_feature_value(const int32_t *ii, int W, const int32_t *d)
{
    const int t = d[0], x = d[1], y = d[2], cw = d[3], ch = d[4];
    switch (t) {
    case 0: /* three-rect horizontal */
        return rect_sum(ii, W, x + cw, y, cw, ch)
             - rect_sum(ii, W, x, y, cw, ch)
             - rect_sum(ii, W, x + 2 * cw, y, cw, ch);
    case 1: /* three-rect vertical */
        return rect_sum(ii, W, x, y + ch, cw, ch)
             - rect_sum(ii, W, x, y, cw, ch)
             - rect_sum(ii, W, x, y + 2 * ch, cw, ch);
    case 2: /* two-rect horizontal */
        return rect_sum(ii, W, x + cw, y, cw, ch)
             - rect_sum(ii, W, x, y, cw, ch);
    case 3: /* two-rect vertical */
        return rect_sum(ii, W, x, y + ch, cw, ch)
             - rect_sum(ii, W, x, y, cw, ch);
    default: /* four-rect */
        return rect_sum(ii, W, x + cw, y, cw, ch)
             + rect_sum(ii, W, x, y + ch, cw, ch)
             - rect_sum(ii, W, x, y, cw, ch)
             - rect_sum(ii, W, x + cw, y + ch, cw, ch);
    }
}

/* All integral images of a window stack: ii_out [N][(H+1)(W+1)]. */
void or_integrals(const uint8_t *images, int64_t N, int W, int H, int32_t *ii_out, int threads)
{
    const int64_t P = (int64_t)(W + 1) * (H + 1);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < N; ++i)
        or_integral(images + i * (int64_t)W * H, W, H, ii_out + i * P);
}

/* Feature values of nf features on all N windows: out [nf][N] (feature-major). */
void or_feature_values(const int32_t *ii, int64_t N, int W, int H,
                       const int32_t *feats, int64_t nf, int32_t *out, int threads)
{
    const int64_t P = (int64_t)(W + 1) * (H + 1);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t j = 0; j < nf; ++j)
        for (int64_t i = 0; i < N; ++i)
            out[j * N + i] = or_feature_value(ii + i * P, W, feats + 5 * j);
}

/* ------------------------------------------------ ordering of one feature
 * Samples sorted by (value, index); a library sort serves as the step. */
typedef struct { int32_t v; int32_t i; } vi_pair;

static int cmp_vi(const void *a, const void *b)
{
    const vi_pair *p = (const vi_pair *)a, *q = (const vi_pair *)b;
    if (p->v != q->v) return p->v < q->v ? -1 : 1;
    return p->i < q->i ? -1 : (p->i > q->i);
}

/* order_out [nf][N]: sample indices of each feature sorted by (value, index). */
void or_sort_features(const int32_t *vals, int64_t N, int64_t nf, int32_t *order_out, int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
#endif
    {
        vi_pair *buf = (vi_pair *)malloc(sizeof(vi_pair) * (size_t)N);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t j = 0; j < nf; ++j) {
            const int32_t *v = vals + j * N;
            for (int64_t i = 0; i < N; ++i) { buf[i].v = v[i]; buf[i].i = (int32_t)i; }
            qsort(buf, (size_t)N, sizeof(vi_pair), cmp_vi);
            for (int64_t i = 0; i < N; ++i) order_out[j * N + i] = buf[i].i;
        }
        free(buf);
    }
}

/* ------------------------------------------------ best stump of one feature
 * Section 2.3 step 2 / Section 3.3.2 step 3a: the stump restricted to one
 * feature with the smallest weighted error
 *     e(p, theta) = sum_i w_i |h(x_i, f, p, theta) - y_i|,
 * h = 1 iff p f(x) < p theta (Section 2.2).
 *
 * With the samples sorted by value, every integer theta predicts "1" for a
 * prefix of the order (p = +1: values below theta) or for a suffix
 * (p = -1: values above theta).  A prefix of length k is realisable only when
 * it does not split a run of equal values: k = 0, k = N, or v_(k) < v_(k+1).
 * For such k, with S+_k / S-_k the weight of positives / negatives among the
 * first k and T+ / T- the totals:
 *     e(+1, k) = S-_k + (T+ - S+_k)     (first k predicted 1)
 *     e(-1, k) = S+_k + (T- - S-_k)     (first k predicted 0)
 * Ties: p = +1 before p = -1, then the smaller k (a reading; the paper is
 * silent).  The threshold is an integer that realises the split:
 *     p = +1: theta = v_(k+1), or v_(N) + 1 when k = N;
 *     p = -1: theta = v_(k),   or v_(1) - 1 when k = 0.
 * Outputs: best error for each polarity (err2[0] for +1, err2[1] for -1) and
 * the overall best (p, k, theta). */
typedef struct {
    double err_pos, err_neg;   /* minimum over k for p = +1 and p = -1 */
    double err;                /* min of the two */
    int32_t polarity;          /* +1 or -1 */
    int32_t split;             /* k */
    int32_t theta;
    int32_t pad;
} or_stump;

static void best_stump_sorted(const int32_t *v, const int32_t *order, const uint8_t *y,
                              const double *w, int64_t N, or_stump *out)
{
    double Tp = 0.0, Tn = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        if (y[i]) Tp += w[i]; else Tn += w[i];
    }
    double Sp = 0.0, Sn = 0.0;
    /* k = 0 */
    double best_pos = Sn + (Tp - Sp); int64_t k_pos = 0;
    double best_neg = Sp + (Tn - Sn); int64_t k_neg = 0;
    for (int64_t k = 1; k <= N; ++k) {
        const int32_t i = order[k - 1];
        if (y[i]) Sp += w[i]; else Sn += w[i];
        const int boundary = (k == N) || (v[order[k - 1]] < v[order[k]]);
        if (!boundary) continue;
        const double ep = Sn + (Tp - Sp);
        const double en = Sp + (Tn - Sn);
        if (ep < best_pos) { best_pos = ep; k_pos = k; }
        if (en < best_neg) { best_neg = en; k_neg = k; }
    }
    out->err_pos = best_pos;
    out->err_neg = best_neg;
    if (best_pos <= best_neg) {
        out->err = best_pos; out->polarity = 1; out->split = (int32_t)k_pos;
        out->theta = (k_pos < N) ? v[order[k_pos]] : v[order[N - 1]] + 1;
    } else {
        out->err = best_neg; out->polarity = -1; out->split = (int32_t)k_neg;
        out->theta = (k_neg > 0) ? v[order[k_neg - 1]] : v[order[0]] - 1;
    }
    out->pad = 0;
}

void or_best_stumps(const int32_t *vals, const int32_t *order, const uint8_t *y,
                    const double *w, int64_t N, int64_t nf, or_stump *out, int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t j = 0; j < nf; ++j)
        best_stump_sorted(vals + j * N, order + j * N, y, w, N, out + j);
}

/* Weak classifier, Section 2.2: 1 iff p f < p theta. */
static int stump_h(int32_t f, int32_t p, int32_t theta)
{
    return (int64_t)p * f < (int64_t)p * theta ? 1 : 0;
}

/* ------------------------------------------------ one boosting round
 * Section 2.3 steps 1-4 (and steps 1 and 4 of the Section 3.3.2 master loop):
 *   1. w <- w / sum(w);
 *   2. every feature's best stump;
 *   3. the stump with the smallest error, ties to the smaller feature index;
 *   4. e_i = 1 if x_i is misclassified, beta = eps / (1 - eps),
 *      w_i <- w_i * beta^(1 - e_i).
 * Reading for eps = 0 (the paper is silent; beta would be 0 and alpha
 * infinite): beta and alpha use eps' = max(eps, eps_floor); the raw eps is
 * reported.  alpha = log(1 / beta), natural log (the base does not change the
 * strong classifier).
 * w is updated in place; the chosen stump goes to *rec. */
typedef struct {
    int64_t feature;
    int32_t polarity, theta, split, pad;
    double err_raw, err, beta, alpha;
    double t_pos, t_neg;    /* class totals of the normalised weights */
} or_round_rec;

int or_round(const int32_t *vals, const int32_t *order, const uint8_t *y, double *w,
             int64_t N, int64_t nf, double eps_floor, or_stump *scratch,
             or_round_rec *rec, int threads)
{
    /* 1. normalise */
    double sum = 0.0;
    for (int64_t i = 0; i < N; ++i) sum += w[i];
    if (!(sum > 0.0)) return -1;
    for (int64_t i = 0; i < N; ++i) w[i] = w[i] / sum;
    double tp = 0.0, tn = 0.0;
    for (int64_t i = 0; i < N; ++i) { if (y[i]) tp += w[i]; else tn += w[i]; }

    /* 2. per-feature best stumps */
    or_best_stumps(vals, order, y, w, N, nf, scratch, threads);

    /* 3. argmin over features */
    int64_t jb = 0;
    for (int64_t j = 1; j < nf; ++j)
        if (scratch[j].err < scratch[jb].err) jb = j;
    const or_stump *s = scratch + jb;

    /* 4. update */
    const double eps = s->err;
    const double epsc = eps > eps_floor ? eps : eps_floor;
    const double beta = epsc / (1.0 - epsc);
    const int32_t *v = vals + jb * N;
    for (int64_t i = 0; i < N; ++i) {
        const int h = stump_h(v[i], s->polarity, s->theta);
        const int e = (h != (int)y[i]);
        if (!e) w[i] = w[i] * beta;   /* beta^(1 - 0); beta^0 = 1 leaves w */
    }
    rec->feature = jb;
    rec->polarity = s->polarity;
    rec->theta = s->theta;
    rec->split = s->split;
    rec->pad = 0;
    rec->err_raw = eps;
    rec->err = epsc;
    rec->beta = beta;
    rec->alpha = log(1.0 / beta);
    rec->t_pos = tp;
    rec->t_neg = tn;
    return 0;
}

/* Initial weights, Section 2.3 Table 2: 1/(2l) for positives, 1/(2m) for
 * negatives.  Returns -1 when a class is empty (the weights are undefined). */
int or_init_weights(const uint8_t *y, int64_t N, double *w)
{
    int64_t l = 0, m = 0;
    for (int64_t i = 0; i < N; ++i) { if (y[i]) ++l; else ++m; }
    if (l == 0 || m == 0) return -1;
    for (int64_t i = 0; i < N; ++i)
        w[i] = y[i] ? 1.0 / (2.0 * (double)l) : 1.0 / (2.0 * (double)m);
    return 0;
}

/* Strong classifier, Section 2.3: C(x) = 1 iff
 * sum_t alpha_t h_t(x) >= 1/2 sum_t alpha_t.
 * fvals [T][N] holds f_t(x_i) for the chosen features. */
void or_strong_classify(const int32_t *fvals, const int32_t *polarity, const int32_t *theta,
                        const double *alpha, int64_t T, int64_t N, uint8_t *out)
{
    double half = 0.0;
    for (int64_t t = 0; t < T; ++t) half += alpha[t];
    half *= 0.5;
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int64_t t = 0; t < T; ++t)
            if (stump_h(fvals[t * N + i], polarity[t], theta[t])) s += alpha[t];
        out[i] = s >= half ? 1 : 0;
    }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
