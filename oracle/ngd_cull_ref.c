/*
 * CPU re-implementation of the tile cull -- TEST INFRASTRUCTURE.
 *
 * Only the test suite may load this code; the product path never calls it.
 * It pins the GPU cull bit for bit: both sides use only IEEE basic operations
 * (+, -, *, fma, min, max, float->int truncation, one float64 division for
 * the key quantiser) in one fixed order, so equal inputs give equal outputs.
 *
 * The steps follow the culling section of the paper (Sec. 3.2):
 *   Eq. 3  project queries and means on random unit vectors r_j:
 *          q_r = q . r,  m_r = m . r
 *   Eq. 4  project the covariance: sigma_r^2 = r^T V r = |L^T r|^2
 *   Eq. 5  drop a Gaussian when the query projection lies outside the
 *          kappa-sigma interval of the projected Gaussian, for some r
 *   tiles  do the test once per tile of queries, bounding the tile's queries
 *          by their extent: a tile keeps Gaussian i unless, for some j,
 *          [m_rj - kappa sigma_rj, m_rj + kappa sigma_rj] misses [lo_tj, hi_tj].
 *
 * Readings where the paper is silent (each shared with the GPU path):
 *   - kappa comes from a value threshold tau: kappa^2 = 2 ln(1/tau), so a
 *     culled pair has G <= tau at every query of the tile.  Eq. 5's printed
 *     "<" contradicts its gloss ("outside the interval"); the gloss is taken.
 *     Equality keeps the pair.
 *   - The interval test is written without square roots:
 *        dist_j = max(lo_tj - m_rj, m_rj - hi_tj, 0)
 *        keep   iff  dist_j * dist_j <= kappa^2 * sigma_rj^2   for every j
 *     with kappa^2 * sigma^2 rounded once to float32 per (Gaussian, j).
 *   - Queries carry no image, so tiles are formed by ordering the queries in
 *     projection space and cutting the order into runs of `tile`:
 *     tiling 0 (k-d): recursive exact-rank splits on the projection of
 *       largest extent (see kd_split) until runs hold at most `tile` queries,
 *       and inside those runs on to runs of 64 (groups of 64 consecutive
 *       queries in a tile are then compact too);
 *     tiling 1 (Morton): a stable sort (ties by original index) on key_proj
 *       projections quantised to key_bits each over the queries' range, bits
 *       interleaved most-significant first;
 *     tiling 2 (given order): the queries keep the caller's order, for
 *       queries that come with an image laid out tile by tile (the paper's
 *       16 x 16 pixel tiles); the Gaussians are ordered as with tiling 0.
 *     Tile t = ordered queries [t*tile, (t+1)*tile).
 *   - Gaussians are ordered the same way by their projected means (k-d runs
 *     of 64; or the Morton key clamped to the queries' range).  Candidate
 *     lists hold ordered Gaussian positions, ascending; the order does not
 *     change any candidate *set*.
 *
 * Rounding recipe:
 *   q_r, m_r : float32 fma chain over dims 0..n-1 starting from 0
 *   sigma^2  : float64; u_b = fma chain over a=b..n-1 of L_ab r_a, then
 *              fma chain over b of u_b^2; rounded to float32
 *   thr      : float32 product kappa2 * sigma2
 *   scale_j  : (float)((double)2^key_bits / ((double)hi_j - (double)lo_j)),
 *              0 when hi_j <= lo_j
 *   digit    : t = q_r - lo (f32); u = t * scale (f32);
 *              u = min(max(u, 0), 2^bits - 1); digit = (int)u
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CULL_MAX_N 32
#define CULL_MAX_PROJ 32

typedef struct {
    int n, n_proj, tile, key_proj, key_bits;
    int64_t k, q, ntiles, total;
    float kappa2;
    int32_t *perm;      /* q: sorted position -> original query index */
    int32_t *gperm;     /* k: sorted position -> original Gaussian index */
    uint32_t *qkey;     /* q: key of each original query */
    uint32_t *gkey;     /* k: key of each original Gaussian */
    float *qlo, *qhi;   /* n_proj: range of the query projections */
    float *tile_lo;     /* ntiles x n_proj */
    float *tile_hi;     /* ntiles x n_proj */
    float *g_mr;        /* k x n_proj (original order) */
    float *g_thr;       /* k x n_proj (original order) */
    float *q_r;         /* q x n_proj (original order) */
    int64_t *tile_off;  /* ntiles + 1 */
    int32_t *cand;      /* total: sorted Gaussian positions */
    int64_t *g_off;     /* k + 1, by sorted Gaussian position */
    int32_t *g_tiles;   /* total */
} cull_ref;

static int cmp_key_idx(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Stable sort of (key, index): pack key in the high 32 bits and the index in
 * the low bits, so a plain sort of the packed values is stable by index. */
static void stable_sort_by_key(const uint32_t *key, int64_t count, int32_t *order)
{
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(count ? count : 1));
    for (int64_t i = 0; i < count; ++i) tmp[i] = ((uint64_t)key[i] << 32) | (uint64_t)i;
    qsort(tmp, (size_t)count, sizeof(uint64_t), cmp_key_idx);
    for (int64_t i = 0; i < count; ++i) order[i] = (int32_t)(tmp[i] & 0xffffffffu);
    free(tmp);
}

/* Order-preserving map of a float to an unsigned key (larger float, larger
 * key; -0 sorts just below +0; NaNs sort above +inf or below -inf). */
static uint32_t orderable(float v)
{
    uint32_t u;
    memcpy(&u, &v, sizeof u);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* k-d ordering: recursively split a run of points (the current order
 * order[lo..hi)) until a run holds at most `sub` points.  A run of n points
 * is cut in units of u = leaf while n > leaf, else of u = sub (sub <= leaf):
 * it needs T = ceil(n/u) units; its first ceil(T/2)*u points in the order
 * (value on the split projection, then current position) go left, the rest
 * right, each side keeping its relative order.  So runs of at most `leaf`
 * points (the tiles) are exactly those of a split with sub = leaf, and the
 * finer splits only reorder points inside them.  The split projection is
 * the one of largest extent (max - min) over the run, the first such on
 * ties. */
static void kd_split(int P, int64_t nall, const float *vals, int32_t *order, int64_t lo,
                     int64_t hi, int leaf, int sub, uint64_t *pairs, int32_t *tmp)
{
    const int64_t n = hi - lo;
    if (n <= sub) return;
    const int64_t u = n > leaf ? leaf : sub;
    const int64_t T = (n + u - 1) / u, nl = ((T + 1) / 2) * u;
    int best = 0;
    float best_ext = 0.0f;
    for (int j = 0; j < P; ++j) {
        float mn = INFINITY, mx = -INFINITY;
        for (int64_t i = lo; i < hi; ++i) {
            const float v = vals[(int64_t)j * nall + order[i]];
            mn = fminf(mn, v);
            mx = fmaxf(mx, v);
        }
        const float ext = mx - mn;
        if (j == 0 || ext > best_ext) {
            best = j;
            best_ext = ext;
        }
    }
    for (int64_t i = lo; i < hi; ++i)
        pairs[i - lo] = ((uint64_t)orderable(vals[(int64_t)best * nall + order[i]]) << 32) |
                        (uint64_t)(i - lo);
    qsort(pairs, (size_t)n, sizeof(uint64_t), cmp_u64);
    const uint64_t pivot = pairs[nl];   /* first point that goes right */
    int64_t l = 0, r = nl;
    for (int64_t i = lo; i < hi; ++i) {
        const uint64_t key =
            ((uint64_t)orderable(vals[(int64_t)best * nall + order[i]]) << 32) | (uint64_t)(i - lo);
        if (key < pivot)
            tmp[l++] = order[i];
        else
            tmp[r++] = order[i];
    }
    memcpy(order + lo, tmp, sizeof(int32_t) * (size_t)n);
    kd_split(P, nall, vals, order, lo, lo + nl, leaf, sub, pairs, tmp);
    kd_split(P, nall, vals, order, lo + nl, hi, leaf, sub, pairs, tmp);
}

static void kd_order(int P, int64_t n, const float *vals, int leaf, int sub, int32_t *order)
{
    for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
    uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    kd_split(P, n, vals, order, 0, n, leaf, sub, pairs, tmp);
    free(pairs);
    free(tmp);
}

static uint32_t morton_key(const float *proj_vals, const float *lo, const float *scale,
                           int key_proj, int key_bits)
{
    const float top = (float)((1u << key_bits) - 1u);
    int digit[CULL_MAX_PROJ];
    for (int j = 0; j < key_proj; ++j) {
        float t = proj_vals[j] - lo[j];
        float u = t * scale[j];
        u = fminf(fmaxf(u, 0.0f), top);
        digit[j] = (int)u;
    }
    uint32_t key = 0;
    for (int b = key_bits - 1; b >= 0; --b)
        for (int j = 0; j < key_proj; ++j)
            key = (key << 1) | (uint32_t)((digit[j] >> b) & 1);
    return key;
}

void ngd_cull_ref_free(cull_ref *c)
{
    if (!c) return;
    free(c->perm); free(c->gperm); free(c->qkey); free(c->gkey);
    free(c->qlo); free(c->qhi); free(c->tile_lo); free(c->tile_hi);
    free(c->g_mr); free(c->g_thr); free(c->q_r); free(c->tile_off); free(c->cand);
    free(c->g_off); free(c->g_tiles);
    free(c);
}

/* Runs the whole cull.  Returns NULL on invalid arguments. */
cull_ref *ngd_cull_ref_run(int n, int64_t k, const float *mean, const float *factor,
                           int64_t q, const float *queries, int n_proj,
                           const float *proj, float kappa2, int tile, int key_proj,
                           int key_bits, int tiling)
{
    if (n < 1 || n > CULL_MAX_N || n_proj < 1 || n_proj > CULL_MAX_PROJ || tile < 1 ||
        key_proj < 0 || key_proj > n_proj || key_bits < 0 || key_proj * key_bits > 32 ||
        k < 0 || q < 0 || tiling < 0 || tiling > 2)
        return NULL;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    cull_ref *c = (cull_ref *)calloc(1, sizeof(cull_ref));
    c->n = n; c->k = k; c->q = q; c->n_proj = n_proj; c->tile = tile;
    c->key_proj = key_proj; c->key_bits = key_bits; c->kappa2 = kappa2;
    c->ntiles = (q + tile - 1) / tile;
    const int64_t T = c->ntiles;
    const size_t kk = (size_t)(k ? k : 1), qq = (size_t)(q ? q : 1);

    /* Eq. 3 for the queries. */
    float *q_r = (float *)malloc(sizeof(float) * qq * n_proj);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < q; ++p)
        for (int j = 0; j < n_proj; ++j) {
            float acc = 0.0f;
            for (int a = 0; a < n; ++a) acc = fmaf(queries[p * n + a], proj[j * n + a], acc);
            q_r[p * n_proj + j] = acc;
        }

    /* Eq. 3 and Eq. 4 for the Gaussians. */
    c->g_mr = (float *)malloc(sizeof(float) * kk * n_proj);
    c->g_thr = (float *)malloc(sizeof(float) * kk * n_proj);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < k; ++i) {
        const float *L = factor + i * tri;
        for (int j = 0; j < n_proj; ++j) {
            const float *r = proj + j * n;
            float acc = 0.0f;
            for (int a = 0; a < n; ++a) acc = fmaf(mean[i * n + a], r[a], acc);
            c->g_mr[i * n_proj + j] = acc;
            double s2 = 0.0;
            for (int b = 0; b < n; ++b) {
                double u = 0.0;   /* (L^T r)_b = sum_{a>=b} L_ab r_a */
                for (int a = b; a < n; ++a)
                    u = fma((double)L[(int64_t)a * (a + 1) / 2 + b], (double)r[a], u);
                s2 = fma(u, u, s2);
            }
            const float s2f = (float)s2;
            c->g_thr[i * n_proj + j] = kappa2 * s2f;
        }
    }

    /* Locality keys over the queries' projected range. */
    c->qlo = (float *)malloc(sizeof(float) * n_proj);
    c->qhi = (float *)malloc(sizeof(float) * n_proj);
    float scale[CULL_MAX_PROJ];
    for (int j = 0; j < n_proj; ++j) {
        float lo = INFINITY, hi = -INFINITY;
        for (int64_t p = 0; p < q; ++p) {
            lo = fminf(lo, q_r[p * n_proj + j]);
            hi = fmaxf(hi, q_r[p * n_proj + j]);
        }
        c->qlo[j] = lo; c->qhi[j] = hi;
        scale[j] = (hi > lo) ? (float)((double)(1u << key_bits) / ((double)hi - (double)lo))
                             : 0.0f;
    }
    c->qkey = (uint32_t *)malloc(sizeof(uint32_t) * qq);
    c->gkey = (uint32_t *)malloc(sizeof(uint32_t) * kk);
    for (int64_t p = 0; p < q; ++p)
        c->qkey[p] = morton_key(q_r + p * n_proj, c->qlo, scale, key_proj, key_bits);
    for (int64_t i = 0; i < k; ++i)
        c->gkey[i] = morton_key(c->g_mr + i * n_proj, c->qlo, scale, key_proj, key_bits);
    c->perm = (int32_t *)malloc(sizeof(int32_t) * qq);
    c->gperm = (int32_t *)malloc(sizeof(int32_t) * kk);
    if (tiling == 0 || tiling == 2) {
        /* k-d order of the query projections (leaves = tiles; tiling 2: the
         * queries keep their given order) and of the projected means (leaves
         * of 64 Gaussians) */
        float *qr_soa = (float *)malloc(sizeof(float) * qq * n_proj);
        for (int64_t p = 0; p < q; ++p)
            for (int j = 0; j < n_proj; ++j) qr_soa[(int64_t)j * q + p] = q_r[p * n_proj + j];
        float *mr_soa = (float *)malloc(sizeof(float) * kk * n_proj);
        for (int64_t i = 0; i < k; ++i)
            for (int j = 0; j < n_proj; ++j) mr_soa[(int64_t)j * k + i] = c->g_mr[i * n_proj + j];
        if (tiling == 0)
            kd_order(n_proj, q, qr_soa, tile, tile < 64 ? tile : 64, c->perm);
        else
            for (int64_t p = 0; p < q; ++p) c->perm[p] = (int32_t)p;
        kd_order(n_proj, k, mr_soa, 64, 64, c->gperm);
        free(qr_soa);
        free(mr_soa);
    } else {
        stable_sort_by_key(c->qkey, q, c->perm);
        stable_sort_by_key(c->gkey, k, c->gperm);
    }

    /* Tile bounds: the extent of each tile's projected queries. */
    c->tile_lo = (float *)malloc(sizeof(float) * (size_t)(T ? T : 1) * n_proj);
    c->tile_hi = (float *)malloc(sizeof(float) * (size_t)(T ? T : 1) * n_proj);
    for (int64_t t = 0; t < T; ++t) {
        const int64_t p0 = t * tile, p1 = (p0 + tile < q) ? p0 + tile : q;
        for (int j = 0; j < n_proj; ++j) {
            float lo = INFINITY, hi = -INFINITY;
            for (int64_t s = p0; s < p1; ++s) {
                const float v = q_r[(int64_t)c->perm[s] * n_proj + j];
                lo = fminf(lo, v);
                hi = fmaxf(hi, v);
            }
            c->tile_lo[t * n_proj + j] = lo;
            c->tile_hi[t * n_proj + j] = hi;
        }
    }

    /* Eq. 5 per (tile, Gaussian), with the per-tile interval. */
    uint8_t *keep = (uint8_t *)malloc((size_t)(T ? T : 1) * kk);
    c->tile_off = (int64_t *)calloc((size_t)(T + 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < T; ++t) {
        int64_t cnt = 0;
        for (int64_t s = 0; s < k; ++s) {
            const int64_t i = c->gperm[s];
            int ok = 1;
            for (int j = 0; j < n_proj && ok; ++j) {
                const float m_r = c->g_mr[i * n_proj + j];
                const float a = c->tile_lo[t * n_proj + j] - m_r;
                const float b = m_r - c->tile_hi[t * n_proj + j];
                const float dist = fmaxf(fmaxf(a, b), 0.0f);
                const float d2 = dist * dist;
                ok = d2 <= c->g_thr[i * n_proj + j];
            }
            keep[t * k + s] = (uint8_t)ok;
            cnt += ok;
        }
        c->tile_off[t + 1] = cnt;
    }
    for (int64_t t = 0; t < T; ++t) c->tile_off[t + 1] += c->tile_off[t];
    c->total = c->tile_off[T];
    c->cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c->total ? c->total : 1));
    int64_t e = 0;
    for (int64_t t = 0; t < T; ++t)
        for (int64_t s = 0; s < k; ++s)
            if (keep[t * k + s]) c->cand[e++] = (int32_t)s;

    /* Transposed lists: for each sorted Gaussian, its tiles in order. */
    c->g_off = (int64_t *)calloc((size_t)(k + 1), sizeof(int64_t));
    c->g_tiles = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c->total ? c->total : 1));
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < k; ++s)
        for (int64_t t = 0; t < T; ++t) c->g_off[s + 1] += keep[t * k + s];
    for (int64_t s = 0; s < k; ++s) c->g_off[s + 1] += c->g_off[s];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < k; ++s) {
        int64_t w = c->g_off[s];
        for (int64_t t = 0; t < T; ++t)
            if (keep[t * k + s]) c->g_tiles[w++] = (int32_t)t;
    }
    free(keep);
    c->q_r = q_r;
    return c;
}

int64_t ngd_cull_ref_total(const cull_ref *c) { return c->total; }
int64_t ngd_cull_ref_ntiles(const cull_ref *c) { return c->ntiles; }

/* Copies the results out; any destination may be NULL. */
void ngd_cull_ref_get(const cull_ref *c, int32_t *perm, int32_t *gperm, int64_t *tile_off,
                      int32_t *cand, int64_t *g_off, int32_t *g_tiles, float *tile_lo,
                      float *tile_hi, float *g_mr, float *g_thr, uint32_t *qkey,
                      uint32_t *gkey, float *qlo, float *qhi, float *q_r)
{
    const int64_t T = c->ntiles, P = c->n_proj;
    if (perm) memcpy(perm, c->perm, sizeof(int32_t) * (size_t)c->q);
    if (gperm) memcpy(gperm, c->gperm, sizeof(int32_t) * (size_t)c->k);
    if (tile_off) memcpy(tile_off, c->tile_off, sizeof(int64_t) * (size_t)(T + 1));
    if (cand) memcpy(cand, c->cand, sizeof(int32_t) * (size_t)c->total);
    if (g_off) memcpy(g_off, c->g_off, sizeof(int64_t) * (size_t)(c->k + 1));
    if (g_tiles) memcpy(g_tiles, c->g_tiles, sizeof(int32_t) * (size_t)c->total);
    if (tile_lo) memcpy(tile_lo, c->tile_lo, sizeof(float) * (size_t)(T * P));
    if (tile_hi) memcpy(tile_hi, c->tile_hi, sizeof(float) * (size_t)(T * P));
    if (g_mr) memcpy(g_mr, c->g_mr, sizeof(float) * (size_t)(c->k * P));
    if (g_thr) memcpy(g_thr, c->g_thr, sizeof(float) * (size_t)(c->k * P));
    if (qkey) memcpy(qkey, c->qkey, sizeof(uint32_t) * (size_t)c->q);
    if (gkey) memcpy(gkey, c->gkey, sizeof(uint32_t) * (size_t)c->k);
    if (qlo) memcpy(qlo, c->qlo, sizeof(float) * (size_t)P);
    if (qhi) memcpy(qhi, c->qhi, sizeof(float) * (size_t)P);
    if (q_r) memcpy(q_r, c->q_r, sizeof(float) * (size_t)(c->q * P));
}
