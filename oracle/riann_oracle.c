/*
 * riann_oracle.c -- plain CPU oracle for RIANN ANN fields.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * library: it has its own patch extraction, distance, table build, integer
 * square root, binary search and reduction, all written in the most direct
 * form, in exact integer arithmetic.
 *
 * Paper: Ben-Zrihem & Zelnik-Manor, "Approximate Nearest Neighbor Fields in
 * Video" (arXiv 1508.07953).
 *
 *   orc_extract     query patches q_{x,y,t}: every p x p (x C) window of a
 *                   frame at stride s, flattened in (dy, dx, c) order
 *                   (Sec. 3.1 notation; 8x8 patches, Sec. 4).
 *   orc_ssd         squared L2 distance between two patches.  The paper's
 *                   dist() is the L2 norm (Sec. 3.1); the square root is
 *                   dropped because it is monotone, and patches are raw
 *                   uint8 (no unit normalisation), so every value is an exact
 *                   integer.
 *   orc_bf          exact nearest neighbour by exhaustive search: the plain
 *                   definition of what the search must return.  Ties go to
 *                   the lowest reference index.
 *   orc_isqrt       floor(sqrt(x)) for x < 2^53, exact.
 *   orc_ring_bounds integer form of the ring test |d(r,k) - d(q,k)| <= R
 *                   (Sec. 3.2, ring of radius d around an anchor; closed
 *                   interval as in Algorithm 1), with R^2 = c.
 *   orc_build       pre-processing (Sec. 3.3): for each key point k, the
 *                   distances from k to every reference patch, sorted
 *                   ascending; plus the n x K pivot table.
 *   orc_riann       the online search of Algorithm 1 in exact mode: the
 *                   radius comes from the previous frame's match and is not
 *                   capped, rings are taken around K fixed key points, the
 *                   smallest ring is scanned and every candidate must lie in
 *                   all K rings; the survivors are checked by exact distance
 *                   and the argmin is returned.
 *   orc_knn_bf      exact k nearest neighbours by exhaustive search, in
 *                   ascending (SSD, index) order.
 *   orc_knn_riann   the same search with k-NN rings: the radius is the
 *                   largest distance to the k previous matches, so the k
 *                   nearest lie inside every ring (exact k-NN fields).
 *   orc_paper       the paper's own approximate search (Algorithm 1): fat
 *                   rings d -/+ alpha*d with alpha = 1/4 around the previous
 *                   match, then around random anchors drawn from the
 *                   candidate set until fewer than L candidates remain.
 *   orc_splitmix    the SplitMix64 generator (Steele, Lea and Flood, 2014)
 *                   that draws the anchors, as a counter-based hash.
 *   orc_extract3d   spatio-temporal query patches (the 3D extension noted in
 *                   Sec. 1): p x p windows of T consecutive frames, flattened
 *                   in (dy, dx, t, c) order.
 *   orc_reconstruct the reconstruction used to judge a field (Sec. 4): every
 *                   query patch is replaced by its match (or by the caller's
 *                   transformed version of that reference, Sec. 5) and
 *                   overlapping patches are averaged; the normalised error
 *                   E = ||f_GT - f_R|| / ||f_GT|| over the covered pixels.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so riann_oracle.c -lm
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF UINT64_MAX

/* Test hook: a non-zero code plants one deliberate mistake so the tests can
 * show that their pins catch it.  Zero (the default) is the correct oracle. */
static int g_fault = 0;
void orc_set_fault(int code) { g_fault = code; }

/* Worker threads of the parallel loops (n <= 0: the OpenMP default); returns
 * the number the next parallel loop will use. */
int orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------ */
/* patches                                                             */
/* ------------------------------------------------------------------ */
void orc_extract(const uint8_t *frame, int H, int W, int C, int64_t pitch,
                 int p, int s, uint8_t *out)
{
    int hq = (H - p) / s + 1, wq = (W - p) / s + 1;
    int D = p * p * C;
    for (int qy = 0; qy < hq; ++qy)
        for (int qx = 0; qx < wq; ++qx) {
            uint8_t *q = out + ((int64_t)qy * wq + qx) * D;
            int y = qy * s, x = qx * s;
            for (int dy = 0; dy < p; ++dy)
                for (int dx = 0; dx < p; ++dx)
                    for (int c = 0; c < C; ++c) {
                        int yy = y + dy, xx = x + dx;
                        if (g_fault == 1) { int t = yy; yy = xx; xx = t; } /* transposed */
                        q[(dy * p + dx) * C + c] =
                            frame[(int64_t)yy * pitch + (int64_t)xx * C + c];
                    }
        }
}

uint64_t orc_ssd(const uint8_t *a, const uint8_t *b, int D)
{
    /* every term is at most 255^2 = 65025, so the sum is exact in 32 bits
     * for D < 66051, far above any patch here */
    const int terms = (g_fault == 2) ? D - 1 : D;        /* planted: dropped term */
    uint32_t s = 0;
    for (int i = 0; i < terms; ++i) {
        const int32_t d = (int32_t)a[i] - (int32_t)b[i];
        s += (uint32_t)(d * d);
    }
    return (uint64_t)s;
}

/* ------------------------------------------------------------------ */
/* exhaustive search                                                   */
/* ------------------------------------------------------------------ */
void orc_bf(const uint8_t *qp, int64_t Q, const uint8_t *ref, int64_t n, int D,
            int32_t *idx, uint32_t *ssd)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < Q; ++i) {
        const uint8_t *q = qp + i * D;
        uint64_t best = ORC_INF;
        int64_t arg = -1;
        for (int64_t r = 0; r < n; ++r) {
            uint64_t d = orc_ssd(q, ref + r * D, D);
            int better = (g_fault == 3) ? (d <= best) : (d < best); /* tie rule */
            if (better) { best = d; arg = r; }
        }
        idx[i] = (int32_t)arg;
        ssd[i] = (uint32_t)(arg < 0 ? 0xFFFFFFFFu : best);
    }
}

/* ------------------------------------------------------------------ */
/* exact ring bounds                                                   */
/* ------------------------------------------------------------------ */
uint64_t orc_isqrt(uint64_t x)
{
    uint64_t s = (uint64_t)sqrt((double)x);
    while (s > 0 && s * s > x) --s;
    while ((s + 1) * (s + 1) <= x) ++s;
    return s;
}

/* Ring of key k for a query: every reference r with
 *     sqrt(b) - sqrt(c) <= sqrt(a) <= sqrt(b) + sqrt(c)
 * where a = SSD(r, k), b = SSD(q, k), c = R^2.  For integer a this is
 *     lo <= a <= hi,  lo = b + c - floor(2 sqrt(bc))  (0 when b <= c),
 *                     hi = b + c + floor(2 sqrt(bc)).
 * c == ORC_INF (no radius) gives the whole table. */
void orc_ring_bounds(uint64_t b, uint64_t c, uint64_t *lo, uint64_t *hi)
{
    if (c == ORC_INF) { *lo = 0; *hi = ORC_INF; return; }
    uint64_t s = orc_isqrt(4 * b * c);
    if (g_fault == 4) s = orc_isqrt(b * c);           /* lost factor 4 */
    *lo = (b <= c) ? 0 : b + c - s;
    if (g_fault == 5) *lo = (b + c > s) ? b + c - s : 0; /* same when b > c */
    if (g_fault == 6 && b <= c) *lo = c - b;          /* wrong sign case */
    *hi = b + c + s;
}

/* ------------------------------------------------------------------ */
/* pre-processing: sorted key-distance tables                           */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t v; int32_t r; } orc_pair;

static int orc_cmp_u64(const void *x, const void *y)
{
    const uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return (a > b) - (a < b);
}

static int orc_cmp_pair(const void *x, const void *y)
{
    const orc_pair *a = (const orc_pair *)x, *b = (const orc_pair *)y;
    if (a->v != b->v) return a->v < b->v ? -1 : 1;
    return (a->r > b->r) - (a->r < b->r);
}

/* T[k*n + j] ascending distances from key k, P[k*n + j] the matching
 * reference index (ties by index), Piv[r*K + k] = SSD(ref_r, ref_{key_k}). */
void orc_build(const uint8_t *ref, int64_t n, int D, const int32_t *keys, int K,
               uint32_t *T, int32_t *P, uint32_t *Piv)
{
    for (int k = 0; k < K; ++k) {
        const uint8_t *kp = ref + (int64_t)keys[k] * D;
        orc_pair *pr = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
        for (int64_t r = 0; r < n; ++r) {
            uint32_t d = (uint32_t)orc_ssd(ref + r * D, kp, D);
            Piv[r * K + k] = d;
            pr[r].v = d;
            pr[r].r = (int32_t)r;
        }
        qsort(pr, (size_t)n, sizeof(orc_pair), orc_cmp_pair);
        for (int64_t j = 0; j < n; ++j) {
            T[(int64_t)k * n + j] = pr[j].v;
            P[(int64_t)k * n + j] = pr[j].r;
        }
        free(pr);
    }
}

/* first j in [0,n) with t[j] >= v */
static int64_t orc_lower(const uint32_t *t, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)t[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* first j in [0,n) with t[j] > v */
static int64_t orc_upper(const uint32_t *t, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)t[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------ */
/* exact-mode RIANN (Algorithm 1 with a key-point ring and uncapped R)  */
/* ------------------------------------------------------------------ */
/* Per query i (patch qp[i*D..]):
 *   c     = SSD(q, ref[prev[i]]), or "no radius" if prev[i] is outside [0,n)
 *   b_k   = SSD(q, ref[keys[k]])
 *   ring k: [lo_k, hi_k] (orc_ring_bounds), located in the sorted table of
 *           key k by two binary searches: [st_k, en_k), m_k = en_k - st_k
 *   k*    = smallest m_k (lowest k on ties)
 *   S     = { P[k*][j], st <= j < en : lo_k <= Piv[r][k] <= hi_k for all k }
 *   out   = (ssd, idx) minimum over S, ties to the lowest index.
 * With K == 0 the candidate set is the whole reference set.
 * Optional per-query outputs (may be NULL): mstar, kstar, nsurv, noprior.
 * With hinted == 1, prev is a hint only (used the same way). */
void orc_riann(const uint8_t *qp, int64_t Q, const uint8_t *ref, int64_t n, int D,
               const int32_t *keys, int K, const uint32_t *T, const int32_t *P,
               const uint32_t *Piv, const int32_t *prev,
               int32_t *idx, uint32_t *ssd, int64_t *mstar, int32_t *kstar,
               int64_t *nsurv, uint8_t *noprior)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < Q; ++i) {
        const uint8_t *q = qp + i * D;
        int32_t pv = prev[i];
        int np = (pv < 0 || (int64_t)pv >= n);
        uint64_t c = np ? ORC_INF : orc_ssd(q, ref + (int64_t)pv * D, D);
        uint64_t *lo = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(K + 1));
        uint64_t *hi = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(K + 1));
        int64_t bst = 0, ben = n, bm = n;
        int bk = -1;
        for (int k = 0; k < K; ++k) {
            uint64_t b = orc_ssd(q, ref + (int64_t)keys[k] * D, D);
            orc_ring_bounds(b, c, &lo[k], &hi[k]);
            const uint32_t *t = T + (int64_t)k * n;
            int64_t st = orc_lower(t, n, lo[k]);
            int64_t en = (hi[k] == ORC_INF) ? n : orc_upper(t, n, hi[k]);
            if (g_fault == 7) en = (hi[k] == ORC_INF) ? n : orc_lower(t, n, hi[k]); /* open end */
            int64_t m = en - st;
            if (bk < 0 || m < bm) { bm = m; bk = k; bst = st; ben = en; }
        }
        uint64_t best = ORC_INF;
        int64_t arg = -1, cnt = 0;
        for (int64_t j = bst; j < ben; ++j) {
            int64_t r = (bk < 0) ? j : P[(int64_t)bk * n + j];
            int in = 1;
            for (int k = 0; k < K && in; ++k) {
                uint64_t a = Piv[r * K + k];
                if (a < lo[k] || a > hi[k]) in = 0;
            }
            if (!in) continue;
            ++cnt;
            uint64_t d = orc_ssd(q, ref + r * D, D);
            if (d < best || (d == best && r < arg)) { best = d; arg = r; }
        }
        idx[i] = (int32_t)arg;
        ssd[i] = (uint32_t)(arg < 0 ? 0xFFFFFFFFu : best);
        if (mstar) mstar[i] = bm;
        if (kstar) kstar[i] = bk;
        if (nsurv) nsurv[i] = cnt;
        if (noprior) noprior[i] = (uint8_t)np;
        free(lo);
        free(hi);
    }
}

/* ------------------------------------------------------------------ */
/* exact k nearest neighbours                                          */
/* ------------------------------------------------------------------ */
/* Insert (d, r) into the ascending list (bd, br) of length kk, keeping the k
 * smallest by (distance, index). */
static void orc_topk_insert(uint64_t *bd, int64_t *br, int kk, uint64_t d, int64_t r)
{
    int pos = kk;
    while (pos > 0 && (d < bd[pos - 1] || (d == bd[pos - 1] && r < br[pos - 1]))) --pos;
    if (pos >= kk) return;
    for (int j = kk - 1; j > pos; --j) { bd[j] = bd[j - 1]; br[j] = br[j - 1]; }
    bd[pos] = d;
    br[pos] = r;
}

/* idx/ssd: Q x k, each row ascending by (SSD, index); k <= n. */
void orc_knn_bf(const uint8_t *qp, int64_t Q, const uint8_t *ref, int64_t n, int D, int k,
                int32_t *idx, uint32_t *ssd)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < Q; ++i) {
        uint64_t bd[64];
        int64_t br[64];
        for (int j = 0; j < k; ++j) { bd[j] = ORC_INF; br[j] = -1; }
        for (int64_t r = 0; r < n; ++r)
            orc_topk_insert(bd, br, k, orc_ssd(qp + i * D, ref + r * D, D), r);
        for (int j = 0; j < k; ++j) {
            idx[i * k + j] = (int32_t)br[j];
            ssd[i * k + j] = (uint32_t)bd[j];
        }
    }
}

/* Exact-mode RIANN for k-NN fields.  prev: Q x k previous matches.  When all
 * k entries are in [0, n) and distinct, the radius c is the largest of their
 * SSDs to the query: those k references lie within sqrt(c), so the k nearest
 * do too, and they are in every ring; otherwise there is no radius.  Rings,
 * the smallest ring and the all-ring filter are as in orc_riann; the answer
 * is the k smallest (SSD, index) over S. */
void orc_knn_riann(const uint8_t *qp, int64_t Q, const uint8_t *ref, int64_t n, int D,
                   const int32_t *keys, int K, const uint32_t *T, const int32_t *P,
                   const uint32_t *Piv, const int32_t *prev, int k, int32_t *idx,
                   uint32_t *ssd)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < Q; ++i) {
        const uint8_t *q = qp + i * D;
        int np = 0;
        uint64_t c = 0;
        for (int j = 0; j < k && !np; ++j) {
            const int32_t pv = prev[i * k + j];
            if (pv < 0 || (int64_t)pv >= n) { np = 1; break; }
            for (int j2 = 0; j2 < j; ++j2)
                if (prev[i * k + j2] == pv) np = 1;
            const uint64_t d = orc_ssd(q, ref + (int64_t)pv * D, D);
            if (g_fault == 10) { if (j == 0 || d < c) c = d; }   /* planted: min, not max */
            else if (d > c) c = d;
        }
        if (np) c = ORC_INF;
        uint64_t *lo = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(K + 1));
        uint64_t *hi = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(K + 1));
        int64_t bst = 0, ben = n, bm = n;
        int bk = -1;
        for (int kk = 0; kk < K; ++kk) {
            uint64_t b = orc_ssd(q, ref + (int64_t)keys[kk] * D, D);
            orc_ring_bounds(b, c, &lo[kk], &hi[kk]);
            const uint32_t *t = T + (int64_t)kk * n;
            int64_t st = orc_lower(t, n, lo[kk]);
            int64_t en = (hi[kk] == ORC_INF) ? n : orc_upper(t, n, hi[kk]);
            int64_t m = en - st;
            if (bk < 0 || m < bm) { bm = m; bk = kk; bst = st; ben = en; }
        }
        uint64_t bd[64];
        int64_t br[64];
        for (int j = 0; j < k; ++j) { bd[j] = ORC_INF; br[j] = -1; }
        for (int64_t j = bst; j < ben; ++j) {
            int64_t r = (bk < 0) ? j : P[(int64_t)bk * n + j];
            int in = 1;
            for (int kk = 0; kk < K && in; ++kk) {
                uint64_t a = Piv[r * K + kk];
                if (a < lo[kk] || a > hi[kk]) in = 0;
            }
            if (in) orc_topk_insert(bd, br, k, orc_ssd(q, ref + r * D, D), r);
        }
        for (int j = 0; j < k; ++j) {
            idx[i * k + j] = (int32_t)br[j];
            ssd[i * k + j] = (uint32_t)(br[j] < 0 ? 0xFFFFFFFFu : bd[j]);
        }
        free(lo);
        free(hi);
    }
}

/* ------------------------------------------------------------------ */
/* the paper's approximate search (Algorithm 1)                        */
/* ------------------------------------------------------------------ */
/* SplitMix64 output for state x: add the golden gamma, then two
 * xor-shift-multiply rounds and a final xor-shift. */
uint64_t orc_splitmix(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The anchor draw of (seed, frame t, query, iteration): a chain of SplitMix64
 * steps, one counter mixed in per step. */
static uint64_t orc_draw(uint64_t seed, uint64_t t, uint64_t query, uint64_t it)
{
    return orc_splitmix(orc_splitmix(orc_splitmix(orc_splitmix(seed) ^ t) ^ query) ^ it);
}

/* With alpha = 1/4 the ring d - alpha d <= dist(r_k, r_j) <= d + alpha d
 * reads, in squared integer distances a = SSD(r_k, r_j) and c = d^2,
 * 9c <= 16a <= 25c. */
static int orc_in_fat_ring(uint64_t a, uint64_t c)
{
    if (g_fault == 11) return 9 * c < 16 * a && 16 * a < 25 * c;   /* planted: open ends */
    return 9 * c <= 16 * a && 16 * a <= 25 * c;
}

/* dm: n x n SSD matrix between references; tv/tp: each row of dm sorted
 * ascending by (value, index) -- values and indices.  Per query i (global
 * index qbase + i within frame t):
 *   r_i = prev[i] (outside [0,n): a random initial match, the draw with
 *         iteration 2^32 - 1, modulo n)
 *   c   = SSD(q, r_i);  S = ring of r_i (positions of its sorted row with
 *         9c <= 16a <= 25c), in row order, preceded by r_i itself when c > 0
 *         (its own ring excludes it otherwise)
 *   while |S| >= L and some member of S has not been an anchor:
 *       u = draw(iteration) mod (number of members not yet anchors); the
 *       anchor r_k is the u-th such member in S order; S' = members of S in
 *       the ring of r_k (radius from SSD(q, r_k)); if S' is empty stop
 *       (keep S), else S = S'
 *   out = (SSD, index) minimum over S.
 * iters (optional): anchors drawn per query. */
void orc_paper(const uint8_t *qp, int64_t Q, const uint8_t *ref, int64_t n, int D,
               const uint32_t *dm, const uint32_t *tv, const int32_t *tp, const int32_t *prev,
               int L, uint64_t seed, uint64_t t, int64_t qbase, int32_t *idx, uint32_t *ssd,
               int32_t *iters)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < Q; ++i) {
        const uint8_t *q = qp + i * D;
        int64_t ri = prev[i];
        if (ri < 0 || ri >= n)
            ri = (int64_t)(orc_draw(seed, t, (uint64_t)(qbase + i), 0xFFFFFFFFull) % (uint64_t)n);
        const uint64_t c = orc_ssd(q, ref + ri * D, D);
        /* ring of r_i in its sorted row */
        const uint32_t *row = tv + ri * n;
        int64_t st = 0, en = 0;
        while (st < n && !(16 * (uint64_t)row[st] >= 9 * c && (g_fault != 11 || 16 * (uint64_t)row[st] > 9 * c))) ++st;
        en = st;
        while (en < n && orc_in_fat_ring(row[en], c)) ++en;
        /* S as a list of reference indices in S order, with anchor marks */
        int64_t cap = (en - st) + 1, m = 0;
        int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        uint8_t *used = (uint8_t *)calloc((size_t)cap, 1);
        int64_t *S2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        uint8_t *used2 = (uint8_t *)malloc((size_t)cap);
        if (c > 0) S[m++] = ri;
        for (int64_t pos = st; pos < en; ++pos) S[m++] = tp[ri * n + pos];
        int32_t it = 0;
        for (;;) {
            if (m < L) break;
            int64_t free_cnt = 0;
            for (int64_t e = 0; e < m; ++e) free_cnt += !used[e];
            if (free_cnt == 0) break;
            const uint64_t u = orc_draw(seed, t, (uint64_t)(qbase + i), (uint64_t)it) %
                               (uint64_t)free_cnt;
            int64_t e = 0, seen = 0;
            for (; e < m; ++e)
                if (!used[e]) {
                    if ((uint64_t)seen == u) break;
                    ++seen;
                }
            used[e] = 1;
            ++it;
            const int64_t rk = S[e];
            /* the anchor's ring: radius d_k = dist(q, r_k), distances from r_k */
            const uint64_t ck = (g_fault == 12) ? c                  /* planted: radius d_i */
                                                : orc_ssd(q, ref + rk * D, D);
            const int64_t rrow = (g_fault == 13) ? ri : rk;          /* planted: r_i's row */
            int64_t m2 = 0;
            for (int64_t f = 0; f < m; ++f)
                if (orc_in_fat_ring(dm[rrow * n + S[f]], ck)) {
                    S2[m2] = S[f];
                    used2[m2] = used[f];
                    ++m2;
                }
            if (m2 == 0) break;
            memcpy(S, S2, sizeof(int64_t) * (size_t)m2);
            memcpy(used, used2, (size_t)m2);
            m = m2;
        }
        uint64_t best = ORC_INF;
        int64_t arg = -1;
        for (int64_t e = 0; e < m; ++e) {
            const uint64_t d = orc_ssd(q, ref + S[e] * D, D);
            if (d < best || (d == best && S[e] < arg)) { best = d; arg = S[e]; }
        }
        if (m == 0) { arg = ri; best = c; }   /* empty ring of r_i and c == 0 cannot happen */
        idx[i] = (int32_t)arg;
        ssd[i] = (uint32_t)best;
        if (iters) iters[i] = it;
        free(S); free(used); free(S2); free(used2);
    }
}

/* Pairwise SSD matrix of the references and its rows sorted by (value,
 * index): the paper's pre-processing for Algorithm 1 (Sec. 3.3). */
void orc_paper_tables(const uint8_t *ref, int64_t n, int D, uint32_t *dm, uint32_t *tv,
                      int32_t *tp)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t *pr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
        for (int64_t j = 0; j < n; ++j) {
            const uint32_t d = (uint32_t)orc_ssd(ref + i * D, ref + j * D, D);
            dm[i * n + j] = d;
            pr[j] = ((uint64_t)d << 32) | (uint64_t)j;
        }
        qsort(pr, (size_t)n, sizeof(uint64_t), orc_cmp_u64);
        for (int64_t j = 0; j < n; ++j) {
            tv[i * n + j] = (uint32_t)(pr[j] >> 32);
            tp[i * n + j] = (int32_t)(pr[j] & 0xFFFFFFFFu);
        }
        free(pr);
    }
}

/* Candidate set S of one query, in scan order (for tests of the
 * containment property).  Returns |S|; writes at most cap indices. */
int64_t orc_riann_candidates(const uint8_t *q, const uint8_t *ref, int64_t n, int D,
                             const int32_t *keys, int K, const uint32_t *T,
                             const int32_t *P, const uint32_t *Piv, int32_t prev,
                             int32_t *out, int64_t cap)
{
    int np = (prev < 0 || (int64_t)prev >= n);
    uint64_t c = np ? ORC_INF : orc_ssd(q, ref + (int64_t)prev * D, D);
    uint64_t lo[1024], hi[1024];
    if (K > 1024) return -1;
    int64_t bst = 0, ben = n, bm = n;
    int bk = -1;
    for (int k = 0; k < K; ++k) {
        uint64_t b = orc_ssd(q, ref + (int64_t)keys[k] * D, D);
        orc_ring_bounds(b, c, &lo[k], &hi[k]);
        const uint32_t *t = T + (int64_t)k * n;
        int64_t st = orc_lower(t, n, lo[k]);
        int64_t en = (hi[k] == ORC_INF) ? n : orc_upper(t, n, hi[k]);
        if (bk < 0 || en - st < bm) { bm = en - st; bk = k; bst = st; ben = en; }
    }
    int64_t cnt = 0;
    for (int64_t j = bst; j < ben; ++j) {
        int64_t r = (bk < 0) ? j : P[(int64_t)bk * n + j];
        int in = 1;
        for (int k = 0; k < K && in; ++k) {
            uint64_t a = Piv[r * K + k];
            if (a < lo[k] || a > hi[k]) in = 0;
        }
        if (!in) continue;
        if (cnt < cap) out[cnt] = (int32_t)r;
        ++cnt;
    }
    return cnt;
}

/* frames: T separate H x W x C frames (oldest first), each with row pitch
 * W*C; out: Hq*Wq patches of p*p*T*C bytes in (dy, dx, t, c) order. */
void orc_extract3d(const uint8_t *const *frames, int T, int H, int W, int C, int p, int s,
                   uint8_t *out)
{
    int hq = (H - p) / s + 1, wq = (W - p) / s + 1;
    int64_t D = (int64_t)p * p * T * C;
    for (int qy = 0; qy < hq; ++qy)
        for (int qx = 0; qx < wq; ++qx) {
            uint8_t *q = out + ((int64_t)qy * wq + qx) * D;
            int64_t k = 0;
            for (int dy = 0; dy < p; ++dy)
                for (int dx = 0; dx < p; ++dx)
                    for (int t = 0; t < T; ++t)
                        for (int c = 0; c < C; ++c) {
                            int tt = (g_fault == 9) ? T - 1 - t : t;   /* planted: time reversed */
                            q[k++] = frames[tt][((int64_t)(qy * s + dy) * W + (qx * s + dx)) * C + c];
                        }
        }
}

/* ------------------------------------------------------------------ */
/* reconstruction (Sec. 4) and patch replacement (Sec. 5)              */
/* ------------------------------------------------------------------ */
/* field: hq x wq match indices; app: n x (p*p*Ca) appearance patches in
 * (dy, dx, c) order (the references themselves, or their transformed
 * versions).  A field entry outside [0, n) names no reference and
 * contributes no patch.  Outputs per pixel of the H x W x Ca frame: the sum of the
 * covering patches' values and how many patches cover it; f_R = sum / count
 * as float32 (0 where nothing covers).  If gt (H x W x Ca, row pitch
 * W*Ca) is given, err[0] = E, err[1] = sum (gt - f_R)^2, err[2] = sum gt^2,
 * err[3] = number of covered values, all over covered pixels only. */
void orc_reconstruct(const int32_t *field, int hq, int wq, const uint8_t *app, int64_t n, int p,
                     int Ca, int s, int H, int W, uint32_t *sum, uint32_t *count, float *fr,
                     const uint8_t *gt, double *err)
{
    const int64_t npx = (int64_t)H * W;
    memset(sum, 0, sizeof(uint32_t) * npx * Ca);
    memset(count, 0, sizeof(uint32_t) * npx);
    for (int i = 0; i < hq; ++i)
        for (int j = 0; j < wq; ++j) {
            const int64_t r = field[(int64_t)i * wq + j];
            if (r < 0 || r >= n) continue;
            const uint8_t *patch = app + r * p * p * Ca;
            for (int dy = 0; dy < p; ++dy)
                for (int dx = 0; dx < p; ++dx) {
                    const int64_t px = (int64_t)(s * i + dy) * W + (s * j + dx);
                    count[px] += 1;
                    for (int c = 0; c < Ca; ++c)
                        sum[px * Ca + c] += patch[(dy * p + dx) * Ca + c];
                }
        }
    double se = 0.0, sg = 0.0, nv = 0.0;
    for (int64_t px = 0; px < npx; ++px)
        for (int c = 0; c < Ca; ++c) {
            const int64_t v = px * Ca + c;
            if (count[px] == 0) { fr[v] = 0.0f; continue; }
            fr[v] = (float)sum[v] / (float)count[px];
            if (gt) {
                const double g = (double)gt[v];
                const double d = g - (double)fr[v];
                se += (g_fault == 8) ? d : d * d;          /* planted: unsquared error */
                sg += g * g;
                nv += 1.0;
            }
        }
    if (gt && err) {
        err[0] = sg > 0.0 ? sqrt(se / sg) : 0.0;
        err[1] = se;
        err[2] = sg;
        err[3] = nv;
    }
}
