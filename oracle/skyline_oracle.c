/*
 * skyline_oracle.c -- CPU oracle for the partitioned skyline method.
 *
 * TEST INFRASTRUCTURE ONLY. This file is a plain, slow, obviously correct CPU
 * implementation used by the tests, by the package's smoke check and by the
 * benchmark's CPU-baseline column. The GPU library never links, loads or calls
 * it, and it shares no source, header, table or helper with the GPU path.
 *
 * Paper: P. Ciaccia, D. Martinenghi, "Optimization Strategies for Parallel
 * Computation of Skylines" (arXiv 2411.14968). Citations name the paper's
 * sections, definitions, algorithms, propositions and equations.
 *
 * Conventions (readings of the paper, stated once here and in the design notes):
 *  - Points are float32, SoA layout: coordinate k of point i is pts[k*n + i].
 *  - Smaller is better in every dimension (Section 2, the convention after Def. 1).
 *  - The input is a multiset indexed 0..n-1; exact duplicates never dominate each
 *    other, so all copies of a point share one fate.
 *  - Scores that decide an integer (the Sorted representatives) are the float32
 *    sequential sum x0 + x1 + ... , evaluated in that order without contraction,
 *    which is the precision the GPU path takes the same decision in.
 *  - Everything else is exact: dominance is a comparison, partition formulas are
 *    evaluated in float64 where they involve arithmetic.
 *
 * Pins: every function here is checked by the not-gpu tests against closed forms,
 * brute force on tiny inputs, invariants and independent algorithms; the MLP
 * gradient is pinned by central finite differences.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PT(pts, n, k, i) ((pts)[(int64_t)(k) * (n) + (i)])

/* ------------------------------------------------------------------------ */
/* Def. 1 (Section 2): t dominates s iff t[A] <= s[A] for every attribute and */
/* t[A'] < s[A'] for at least one.                                          */
/* ------------------------------------------------------------------------ */
static int dom_soa(const float *pts, int64_t n, int d, int64_t t, int64_t s)
{
    int strict = 0;
    for (int k = 0; k < d; ++k) {
        float a = PT(pts, n, k, t), b = PT(pts, n, k, s);
        if (a > b) return 0;
        if (a < b) strict = 1;
    }
    return strict;
}

/* Same test on two points given as contiguous coordinate vectors. */
static int dom_vec(const float *t, const float *s, int d)
{
    int strict = 0;
    for (int k = 0; k < d; ++k) {
        if (t[k] > s[k]) return 0;
        if (t[k] < s[k]) strict = 1;
    }
    return strict;
}

/* ------------------------------------------------------------------------ */
/* O1: brute force -- the skyline definition (Def. 1) written out.           */
/* in_sky[i] = 1 iff no j dominates i. Returns |Sky|.                        */
/* ------------------------------------------------------------------------ */
int64_t or_sky_brute(const float *pts, int64_t n, int32_t d, uint8_t *in_sky)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        int dominated = 0;
        for (int64_t j = 0; j < n && !dominated; ++j)
            if (j != i && dom_soa(pts, n, d, j, i)) dominated = 1;
        in_sky[i] = (uint8_t)!dominated;
        cnt += !dominated;
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* O2: exact 2-D skyline by sort and scan (the textbook low-dimensional      */
/* method the introduction cites). Sort by (x, y, id); within a group of      */
/* equal x only the copies of the group's minimum y can survive, and they do */
/* iff that minimum is below every y seen in groups with smaller x.          */
/* ------------------------------------------------------------------------ */
typedef struct { float x, y; int64_t id; } xy_t;

static int cmp_xy(const void *a, const void *b)
{
    const xy_t *p = a, *q = b;
    if (p->x < q->x) return -1;
    if (p->x > q->x) return 1;
    if (p->y < q->y) return -1;
    if (p->y > q->y) return 1;
    return (p->id > q->id) - (p->id < q->id);
}

int64_t or_sky_2d(const float *pts, int64_t n, uint8_t *in_sky)
{
    xy_t *v = malloc(sizeof(xy_t) * (size_t)(n > 0 ? n : 1));
    if (!v) return -1;
    for (int64_t i = 0; i < n; ++i) {
        v[i].x = PT(pts, n, 0, i);
        v[i].y = PT(pts, n, 1, i);
        v[i].id = i;
        in_sky[i] = 0;
    }
    qsort(v, (size_t)n, sizeof(xy_t), cmp_xy);
    int64_t cnt = 0;
    float best_before = INFINITY; /* min y over groups with strictly smaller x */
    for (int64_t g = 0; g < n;) {
        int64_t e = g;
        while (e < n && v[e].x == v[g].x) ++e;
        float gmin = v[g].y;
        for (int64_t i = g; i < e; ++i)
            if (v[i].y == gmin && gmin < best_before) { in_sky[v[i].id] = 1; ++cnt; }
        if (gmin < best_before) best_before = gmin;
        g = e;
    }
    free(v);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* O3: SFS (Algorithm 1). The monotone function is the lexicographic key     */
/* (float64 sum of the coordinates, x0, ..., x_{d-1}, id), a linear           */
/* extension of dominance: if s dominates t the sum of s is not larger and,  */
/* on equal sums, s is lexicographically smaller.                            */
/* Works on an index subset `idx` (len m) of the SoA array; writes keep[j]    */
/* for idx[j]. Counts dominance tests (window scan stops at the first        */
/* dominator). Returns the number kept.                                      */
/* ------------------------------------------------------------------------ */
typedef struct { const float *pts; int64_t n; int d; const double *sum; } sfs_ctx;

static int cmp_sfs(const void *a, const void *b, void *arg)
{
    const sfs_ctx *c = arg;
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (c->sum[i] < c->sum[j]) return -1;
    if (c->sum[i] > c->sum[j]) return 1;
    for (int k = 0; k < c->d; ++k) {
        float x = PT(c->pts, c->n, k, i), y = PT(c->pts, c->n, k, j);
        if (x < y) return -1;
        if (x > y) return 1;
    }
    return (i > j) - (i < j);
}

static double sum64(const float *pts, int64_t n, int d, int64_t i)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += (double)PT(pts, n, k, i);
    return s;
}

/* SFS over the subset idx[0..m) (Algorithm 1, Section 2). sums[] is indexed by
 * point id. Visiting the points in an order that never puts a point after one
 * it dominates (cmp_sfs), a point belongs to the skyline of the subset exactly
 * when none of the skyline points met before it dominates it: a dominator of
 * a point is met earlier, and a dominated dominator is itself dominated by an
 * earlier skyline point (transitivity). So each point is compared with the
 * skyline found so far, in the order it was found, until one dominates it.
 * keep_by_id[t] is set for every t of the subset; `tests` accumulates the
 * comparisons; order_out (nullable) receives the skyline ids in visit order.
 * Returns the skyline size. */
static int64_t sfs_subset(const float *pts, int64_t n, int d, const double *sums,
                          const int64_t *idx, int64_t m, uint8_t *keep_by_id, int64_t *tests,
                          int64_t *order_out)
{
    if (m <= 0) return 0;
    int64_t *visit = malloc(sizeof(int64_t) * (size_t)m);
    float *sky = malloc(sizeof(float) * (size_t)m * (size_t)d);   /* coordinates of the skyline so far */
    float *cur = malloc(sizeof(float) * (size_t)d);
    memcpy(visit, idx, sizeof(int64_t) * (size_t)m);
    sfs_ctx c = {pts, n, d, sums};
    qsort_r(visit, (size_t)m, sizeof(int64_t), cmp_sfs, &c);
    int64_t found = 0, compared = 0;
    for (int64_t a = 0; a < m; ++a) {
        const int64_t t = visit[a];
        for (int k = 0; k < d; ++k) cur[k] = PT(pts, n, k, t);
        int64_t u = 0;
        while (u < found && !dom_vec(sky + u * d, cur, d)) ++u;
        compared += u < found ? u + 1 : found;
        keep_by_id[t] = (uint8_t)(u == found);
        if (u == found) {
            memcpy(sky + found * d, cur, sizeof(float) * (size_t)d);
            if (order_out) order_out[found] = t;
            ++found;
        }
    }
    free(visit); free(sky); free(cur);
    if (tests) *tests += compared;
    return found;
}

int64_t or_sky_sfs(const float *pts, int64_t n, int32_t d, uint8_t *in_sky, int64_t *tests)
{
    double *sums = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t *idx = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { sums[i] = sum64(pts, n, d, i); idx[i] = i; in_sky[i] = 0; }
    if (tests) *tests = 0;
    int64_t c = sfs_subset(pts, n, d, sums, idx, n, in_sky, tests, NULL);
    free(sums); free(idx);
    return c;
}

/* ------------------------------------------------------------------------ */
/* O4: BNL (block nested loops, cited in Section 2 and Section 6) with an    */
/* unbounded window: an incoming point is dropped if a window point          */
/* dominates it; otherwise it evicts the window points it dominates and      */
/* joins the window. No sort, so an algorithm independent of O3.             */
/* ------------------------------------------------------------------------ */
int64_t or_sky_bnl(const float *pts, int64_t n, int32_t d, uint8_t *in_sky)
{
    int64_t *win = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) in_sky[i] = 0;
    for (int64_t t = 0; t < n; ++t) {
        int dominated = 0;
        for (int64_t u = 0; u < w; ++u)
            if (dom_soa(pts, n, d, win[u], t)) { dominated = 1; break; }
        if (dominated) continue;
        int64_t keep = 0;
        for (int64_t u = 0; u < w; ++u)
            if (!dom_soa(pts, n, d, t, win[u])) win[keep++] = win[u];
        w = keep;
        win[w++] = t;
    }
    for (int64_t u = 0; u < w; ++u) in_sky[win[u]] = 1;
    free(win);
    return w;
}

/* ------------------------------------------------------------------------ */
/* Grid partitioning (Section 3.2): p(t) = sum_i floor(t[A_i] m) m^(i-1).    */
/* Readings: dimension 0 is the least significant digit; per-dimension m_k   */
/* is allowed; a coordinate equal to 1 (floor gives m) is clamped to m-1.    */
/* float32 * small integer is exact in float64, so floor is exact.           */
/* Requires coordinates in [0,1]; returns -3 otherwise.                       */
/* ------------------------------------------------------------------------ */
int32_t or_grid_cells(const float *pts, int64_t n, int32_t d, const int32_t *m, uint32_t *cell)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t idx = 0, mult = 1;
        for (int k = 0; k < d; ++k) {
            double x = (double)PT(pts, n, k, i);
            if (!(x >= 0.0 && x <= 1.0)) return -3;
            double f = floor(x * (double)m[k]);
            int64_t c = (int64_t)f;
            if (c > m[k] - 1) c = m[k] - 1;
            idx += (uint64_t)c * mult;
            mult *= (uint64_t)m[k];
        }
        cell[i] = (uint32_t)idx;
    }
    return 0;
}

/* Per-dimension grid coordinates of a cell index (dimension 0 least significant). */
static void cell_coords(uint64_t idx, int d, const int32_t *m, int32_t *c)
{
    for (int k = 0; k < d; ++k) { c[k] = (int32_t)(idx % (uint64_t)m[k]); idx /= (uint64_t)m[k]; }
}

/* ------------------------------------------------------------------------ */
/* Grid Filtering (Section 3.2, grid dominance): cell c_i grid-dominates c_h  */
/* iff c_i[j] < c_h[j] in every dimension; every point of a cell that is      */
/* grid-dominated by a non-empty cell is discarded. Written as the plain     */
/* double loop over pairs of cells. pruned[i] = 1 for discarded points.       */
/* Returns the number of points kept, or -3 for coordinates outside [0,1].    */
/* ------------------------------------------------------------------------ */
int64_t or_grid_filter(const float *pts, int64_t n, int32_t d, const int32_t *m, uint8_t *pruned)
{
    uint64_t ncell = 1;
    for (int k = 0; k < d; ++k) ncell *= (uint64_t)m[k];
    uint32_t *cell = malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    if (or_grid_cells(pts, n, d, m, cell) != 0) { free(cell); return -3; }
    uint8_t *occ = calloc((size_t)ncell, 1);
    uint8_t *dead = calloc((size_t)ncell, 1);
    for (int64_t i = 0; i < n; ++i) occ[cell[i]] = 1;
    int32_t ci[16], ch[16];
    for (uint64_t h = 0; h < ncell; ++h) {
        if (!occ[h]) continue;
        cell_coords(h, d, m, ch);
        for (uint64_t i = 0; i < ncell && !dead[h]; ++i) {
            if (!occ[i]) continue;
            cell_coords(i, d, m, ci);
            int all_lt = 1;
            for (int k = 0; k < d; ++k) if (!(ci[k] < ch[k])) { all_lt = 0; break; }
            if (all_lt) dead[h] = 1;
        }
    }
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) { pruned[i] = dead[cell[i]]; kept += !pruned[i]; }
    free(cell); free(occ); free(dead);
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Angular partitioning (Section 3.3, Eq. (1)).                              */
/* tan(phi_i) = sqrt(sum_{j>i} x_j^2) / x_i, phi_i in [0, pi/2], and          */
/* p(t) = sum_{i=1}^{d-1} floor(2 phi_i m_i / pi) prod_{j<i} m_j.             */
/* Reading: the digit of angle i is the number of k in 1..m_i-1 with          */
/* phi_i >= k pi / (2 m_i), i.e. floor(2 phi_i m_i / pi) clamped to m_i - 1   */
/* (phi_i = pi/2, which happens for x_i = 0, would give m_i). Because tan is  */
/* increasing on [0, pi/2), phi_i >= a_k  <=>  S_i >= x_i^2 tan^2(a_k), with  */
/* S_i = sum_{j>i} x_j^2. S_i and x_i^2 are formed in float64 in index order, */
/* without contraction; tan^2(a_k) is tan() of a_k = k*pi/(2 m_i), squared.  */
/* The first angle is the least significant digit. m has d-1 entries.         */
/* ------------------------------------------------------------------------ */
int32_t or_angular_cells(const float *pts, int64_t n, int32_t d, const int32_t *m, uint32_t *cell)
{
    if (d < 2) { for (int64_t i = 0; i < n; ++i) cell[i] = 0; return 0; }
    double *T = malloc(sizeof(double) * 64 * (size_t)(d - 1));
    for (int a = 0; a < d - 1; ++a) {
        if (m[a] < 1 || m[a] > 64) { free(T); return -1; }
        for (int k = 1; k < m[a]; ++k) {
            double ang = (double)k * M_PI / (2.0 * (double)m[a]);
            double t = tan(ang);
            T[a * 64 + k] = t * t;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        uint64_t idx = 0, mult = 1;
        for (int a = 0; a < d - 1; ++a) {
            double xi = (double)PT(pts, n, a, i);
            if (!(xi >= 0.0 && xi <= 1.0)) { free(T); return -3; }
            double S = 0.0;
            for (int j = a + 1; j < d; ++j) {
                double xj = (double)PT(pts, n, j, i);
                if (!(xj >= 0.0 && xj <= 1.0)) { free(T); return -3; }
                double sq = xj * xj;
                S = S + sq;
            }
            double x2 = xi * xi;
            int digit = 0;
            for (int k = 1; k < m[a]; ++k) {
                double rhs = x2 * T[a * 64 + k];
                if (S >= rhs) digit = k;
            }
            idx += (uint64_t)digit * mult;
            mult *= (uint64_t)m[a];
        }
        cell[i] = (uint32_t)idx;
    }
    free(T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sliced partitioning (Section 3.4): sort on one dimension s with a tie      */
/* break giving a total order, then the i-th tuple goes to partition          */
/* floor(i p / N) (0-based rank; the printed formula with N-1 in the          */
/* denominator would put the last tuple alone into partition p). Reading of   */
/* the tie break: lexicographic (x_s, then x_0..x_{d-1} without s, then id),  */
/* a linear extension of dominance, which the NoSeq choice pd_i = {u_j: j<i}  */
/* needs (Section 4.2).                                                       */
/* ------------------------------------------------------------------------ */
typedef struct { const float *pts; int64_t n; int d; int s; } lex_ctx;

static int cmp_lex(const void *a, const void *b, void *arg)
{
    const lex_ctx *c = arg;
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    float x = PT(c->pts, c->n, c->s, i), y = PT(c->pts, c->n, c->s, j);
    if (x < y) return -1;
    if (x > y) return 1;
    for (int k = 0; k < c->d; ++k) {
        if (k == c->s) continue;
        x = PT(c->pts, c->n, k, i); y = PT(c->pts, c->n, k, j);
        if (x < y) return -1;
        if (x > y) return 1;
    }
    return (i > j) - (i < j);
}

int32_t or_sliced_cells(const float *pts, int64_t n, int32_t d, int32_t s, int32_t p, uint32_t *cell)
{
    if (s < 0 || s >= d || p < 1) return -1;
    int64_t *ord = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) ord[i] = i;
    lex_ctx c = {pts, n, d, s};
    qsort_r(ord, (size_t)n, sizeof(int64_t), cmp_lex, &c);
    for (int64_t r = 0; r < n; ++r)
        cell[ord[r]] = (uint32_t)((r * (int64_t)p) / n);
    free(ord);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Representative Filtering (Section 4.1).                                    */
/* Sorted representatives: the tuples first in the order of a monotone        */
/* function; reading: the global K smallest by (float32 sequential sum, id).   */
/* ------------------------------------------------------------------------ */
void or_sum_scores(const float *pts, int64_t n, int32_t d, float *score)
{
    for (int64_t i = 0; i < n; ++i) {
        float s = PT(pts, n, 0, i);   /* sequential float32 adds */
        for (int k = 1; k < d; ++k) s = s + PT(pts, n, k, i);
        score[i] = s;
    }
}

typedef struct { float s; int64_t id; } sid_t;

static int cmp_sid(const void *a, const void *b)
{
    const sid_t *p = a, *q = b;
    if (p->s < q->s) return -1;
    if (p->s > q->s) return 1;
    return (p->id > q->id) - (p->id < q->id);
}

/* The k smallest points by (score, id), in that order. Returns the count. */
int64_t or_select_reps(const float *score, int64_t n, int32_t k, int64_t *ids)
{
    sid_t *v = malloc(sizeof(sid_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { v[i].s = score[i]; v[i].id = i; }
    qsort(v, (size_t)n, sizeof(sid_t), cmp_sid);
    int64_t c = n < k ? n : k;
    for (int64_t i = 0; i < c; ++i) ids[i] = v[i].id;
    free(v);
    return c;
}

/* Self-filter: a representative dominated by another representative is
 * discarded before the set is shared (Section 4.1). keep[j] for ids[j]. */
int64_t or_rep_selfilter(const float *pts, int64_t n, int32_t d, const int64_t *ids, int64_t k,
                         uint8_t *keep)
{
    int64_t c = 0;
    for (int64_t a = 0; a < k; ++a) {
        int dominated = 0;
        for (int64_t b = 0; b < k && !dominated; ++b)
            if (b != a && dom_soa(pts, n, d, ids[b], ids[a])) dominated = 1;
        keep[a] = (uint8_t)!dominated;
        c += !dominated;
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Region representatives (Section 4.1): the tuples with the largest volume of */
/* their dominance region on [0,1]^d, V(DR(t)) = prod_i (1 - t[i]). Reading:   */
/* V in float32, the factors multiplied in coordinate order without          */
/* contraction; the score is -V so that the K smallest scores (ties by id)   */
/* are the K largest volumes. Returns -3 when a coordinate lies outside [0,1]. */
/* ------------------------------------------------------------------------ */
int32_t or_region_scores(const float *pts, int64_t n, int32_t d, float *score)
{
    for (int64_t i = 0; i < n; ++i) {
        float v = 1.0f;
        for (int k = 0; k < d; ++k) {
            const float x = PT(pts, n, k, i);
            if (!(x >= 0.0f && x <= 1.0f)) return -3;
            v = v * (1.0f - x);
        }
        score[i] = -v;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Random choices (Random partitioning, Section 3.1; random representatives,  */
/* Section 4.1) draw from SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) in its */
/* counter form: draw i from seed s is the output for state s + (i+1)*gamma.  */
/* ------------------------------------------------------------------------ */
uint64_t or_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The stream of the representatives' draws: seed XOR this word. */
#define OR_REPS_STREAM 0xD1B54A32D192ED03ull

/* Random representatives: a uniform sample of K tuples without replacement, */
/* read as the K smallest of u_i = floor(draw_i / 2^40) * 2^-24 (ties by id). */
void or_random_scores(int64_t n, uint64_t seed, float *score)
{
    for (int64_t i = 0; i < n; ++i)
        score[i] = (float)(or_splitmix64(seed ^ OR_REPS_STREAM, (uint64_t)i) >> 40) * 0x1p-24f;
}

typedef struct { uint32_t key; int64_t id; } kid_t;

static int cmp_kid(const void *a, const void *b)
{
    const kid_t *p = a, *q = b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return (p->id > q->id) - (p->id < q->id);
}

/* Random partitioning: tuples spread at random over p equal-sized partitions. */
/* Reading: rank of (floor(draw_i / 2^32), i) in ascending order, then the   */
/* slice rule floor(rank * p / n) of the Sliced strategy.                     */
int32_t or_random_cells(int64_t n, int32_t p, uint64_t seed, uint32_t *cell)
{
    if (p < 1) return -1;
    kid_t *v = malloc(sizeof(kid_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { v[i].key = (uint32_t)(or_splitmix64(seed, (uint64_t)i) >> 32); v[i].id = i; }
    qsort(v, (size_t)n, sizeof(kid_t), cmp_kid);
    for (int64_t r = 0; r < n; ++r) cell[v[r].id] = (uint32_t)(((__int128)r * p) / n);
    free(v);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dominance counts (Def. 2, dominance region): dc(t) = #{s in S : t dom s}.   */
/* ------------------------------------------------------------------------ */
void or_domcount(const float *pts, int64_t n, int32_t d, const uint32_t *sample, int64_t m,
                 const int64_t *which, int64_t nw, uint32_t *out)
{
    for (int64_t a = 0; a < nw; ++a) {
        int64_t t = which ? which[a] : a;
        uint32_t c = 0;
        for (int64_t j = 0; j < m; ++j)
            if (dom_soa(pts, n, d, t, (int64_t)sample[j])) ++c;
        out[a] = c;
    }
}

/* ------------------------------------------------------------------------ */
/* Reverse dominance counts (Def. 2 read the other way round): out[a] = the   */
/* number of points by[j] that dominate point which[a] (every point when      */
/* which is NULL), e.g. whether a set of representatives prunes a point.     */
/* ------------------------------------------------------------------------ */
void or_domby(const float *pts, int64_t n, int32_t d, const int64_t *by, int64_t m,
              const int64_t *which, int64_t nw, uint32_t *out)
{
    for (int64_t a = 0; a < nw; ++a) {
        const int64_t t = which ? which[a] : a;
        uint32_t c = 0;
        for (int64_t j = 0; j < m; ++j)
            if (dom_soa(pts, n, d, by[j], t)) ++c;
        out[a] = c;
    }
}

/* ------------------------------------------------------------------------ */
/* Training targets of the learned scorer, from dominance counts (Def. 2).    */
/* The residual sample keeps the sample points that no point of reps          */
/* dominates (with reps the set's own Sorted representatives, what the        */
/* coordinate sum already prunes is left out). dc(t) counts the residual      */
/* sample points t dominates, scaled to the whole input by n / m with m the   */
/* size of the full sample, and the target is y(t) = -log1p(dc n / m) /       */
/* log1p(n), in float64: 0 for a point that dominates nothing, -1 for one     */
/* that dominates the whole sample. Returns the residual sample's size.       */
/* ------------------------------------------------------------------------ */
int64_t or_mlp_targets(const float *pts, int64_t n, int32_t d, const int64_t *sample, int64_t m,
                       const int64_t *reps, int64_t nreps, double *y)
{
    int64_t *res = malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t kept = 0;
    for (int64_t j = 0; j < m; ++j) {
        int pruned = 0;
        for (int64_t r = 0; r < nreps && !pruned; ++r) pruned = dom_soa(pts, n, d, reps[r], sample[j]);
        if (!pruned) res[kept++] = sample[j];
    }
    const double scale = m > 0 ? (double)n / (double)m : 0.0, norm = log1p((double)n);
    for (int64_t t = 0; t < n; ++t) {
        int64_t dc = 0;
        for (int64_t j = 0; j < kept; ++j) dc += dom_soa(pts, n, d, t, res[j]);
        y[t] = -log1p((double)dc * scale) / norm;
    }
    free(res);
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Learned representatives: the scorer proposes candidates, a coverage count  */
/* chooses among them (the paper's strong tuples of Section 4.1 ranked by a   */
/* learned score instead of the coordinate sum or the region volume).         */
/* Pool: slots [0, half) hold the half smallest points by (float32 sum, id),  */
/* slots [half, 2 half) the half smallest by (learned score, id); a learned    */
/* candidate already among the sum candidates leaves its slot empty (-1), and */
/* so does a slot past n.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double s; int64_t id; } did_t;

static int cmp_did(const void *a, const void *b)
{
    const did_t *p = a, *q = b;
    if (p->s < q->s) return -1;
    if (p->s > q->s) return 1;
    return (p->id > q->id) - (p->id < q->id);
}

void or_learned_pool(const float *sum_score, const double *lscore, int64_t n, int32_t half, int64_t *pool)
{
    int64_t *ids = malloc(sizeof(int64_t) * (size_t)(half > 0 ? half : 1));
    const int64_t k = or_select_reps(sum_score, n, half, ids);
    for (int32_t j = 0; j < half; ++j) pool[j] = j < k ? ids[j] : -1;
    did_t *v = malloc(sizeof(did_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { v[i].s = lscore[i]; v[i].id = i; }
    qsort(v, (size_t)n, sizeof(did_t), cmp_did);
    for (int32_t j = 0; j < half; ++j) {
        int64_t id = j < n ? v[j].id : -1;
        for (int64_t q = 0; q < k && id >= 0; ++q)
            if (ids[q] == id) id = -1;
        pool[half + j] = id;
    }
    free(ids); free(v);
}

/* Candidate set i (i = 0..4) takes the first R - m_i sum slots and the first */
/* m_i learned slots of the pool, R = min(n_reps, half), m_i = floor(i R / 4).*/
/* The set that dominates the most points of the stride sample              */
/* {floor(s n / M) : 0 <= s < M}, M = min(n, sample_cap), is chosen, the      */
/* smallest i on ties. picked receives its ids (the sum part, then the        */
/* learned part, each in slot order, empty slots skipped); cover (nullable)   */
/* the five coverage counts. Returns the number picked.                       */
int64_t or_learned_mix(const float *pts, int64_t n, int32_t d, const int64_t *pool, int32_t half,
                       int32_t n_reps, int64_t sample_cap, int64_t *picked, int64_t *cover)
{
    const int32_t R = n_reps < half ? n_reps : half;
    const int64_t M = n < sample_cap ? n : sample_cap;
    int best = 0;
    int64_t best_cov = -1;
    for (int i = 0; i < 5; ++i) {
        const int32_t mi = i * R / 4;
        int64_t cov = 0;
        for (int64_t s = 0; s < M; ++s) {
            const int64_t q = (int64_t)(((__int128)s * n) / M);
            int hit = 0;
            for (int32_t k = 0; k < R - mi && !hit; ++k)
                hit = pool[k] >= 0 && dom_soa(pts, n, d, pool[k], q);
            for (int32_t k = 0; k < mi && !hit; ++k)
                hit = pool[half + k] >= 0 && dom_soa(pts, n, d, pool[half + k], q);
            cov += hit;
        }
        if (cover) cover[i] = cov;
        if (cov > best_cov) { best = i; best_cov = cov; }
    }
    const int32_t mb = best * R / 4;
    int64_t c = 0;
    for (int32_t k = 0; k < R - mb; ++k) if (pool[k] >= 0) picked[c++] = pool[k];
    for (int32_t k = 0; k < mb; ++k) if (pool[half + k] >= 0) picked[c++] = pool[half + k];
    return c;
}

/* ------------------------------------------------------------------------ */
/* Sorted representatives taken per partition (Section 4.1: the first tuples */
/* of each partition after sorting). Reading: the ceil(K / np) smallest       */
/* points by (float32 sum, id) of every partition, over all its points,       */
/* partition 0's first, each partition's in that order. Returns the count.    */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t part; float s; int64_t id; } psid_t;

static int cmp_psid(const void *a, const void *b)
{
    const psid_t *p = a, *q = b;
    if (p->part != q->part) return p->part < q->part ? -1 : 1;
    if (p->s < q->s) return -1;
    if (p->s > q->s) return 1;
    return (p->id > q->id) - (p->id < q->id);
}

int64_t or_sorted_part_reps(const float *sum_score, int64_t n, const uint32_t *part, int32_t np, int32_t K,
                            int64_t *ids)
{
    const int64_t kp = np > 0 ? (K + np - 1) / np : 0;
    psid_t *v = malloc(sizeof(psid_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { v[i].part = part[i]; v[i].s = sum_score[i]; v[i].id = i; }
    qsort(v, (size_t)n, sizeof(psid_t), cmp_psid);
    int64_t c = 0;
    for (int64_t a = 0; a < n;) {
        int64_t e = a;
        while (e < n && v[e].part == v[a].part) ++e;
        for (int64_t b = a; b < e && b < a + kp; ++b) ids[c++] = v[b].id;
        a = e;
    }
    free(v);
    return c;
}

/* ------------------------------------------------------------------------ */
/* O5/O6: the paper's pipeline (Algorithm 2 with the options of Sections 3     */
/* and 4), in this order:                                                      */
/*   1. partition ids of all points (Grid, Angular, Sliced or Random formulas), */
/*   2. Grid Filtering on its grid (all points occupy cells),                  */
/*   3. representatives chosen from all points (globally, per partition, or    */
/*      the learned pool and mix), self-filtered, and every remaining point    */
/*      dominated by a kept representative removed,                            */
/*   4. parallel for each partition: local skyline u_i = Sky(r_i') by SFS,      */
/*   5. merge: NoSeq, Sky(r) = union_i Sky_{pd_i}(u_i) (Proposition 2) with      */
/*      pd_i = u_j for j<i (Sliced), c_j <= c_i componentwise, j != i (Grid,     */
/*      the weak grid-dominance superset), every j != i (Angular, Random); or   */
/*      the sequential final round Sky(u) (Algorithm 2, last line).            */
/* Statistics are definitions of sets, independent of evaluation order, except */
/* the test counts, which define the algorithmic work of the method:           */
/*   tests_local: the SFS comparisons of step 4 (each point against the local  */
/*     skyline found so far, in the order found, up to the first dominator);    */
/*   tests_merge: NoSeq: each point t of u_i against the u_j of pd_i, j in       */
/*     ascending order, each u_j in SFS order and only over its points that    */
/*     come before t in that order (a dominator of t always does), up to the   */
/*     first dominator; the final round: the SFS comparisons over u.           */
/* ------------------------------------------------------------------------ */
enum { OR_PART_NONE = 0, OR_PART_GRID = 1, OR_PART_ANGULAR = 2, OR_PART_SLICED = 3, OR_PART_RANDOM = 4 };
enum { OR_REPS_NONE = 0, OR_REPS_SORTED = 1, OR_REPS_SCORES = 2, OR_REPS_REGION = 3, OR_REPS_RANDOM = 4,
       OR_REPS_SORTED_PART = 5, OR_REPS_LEARNED = 6 };
enum { OR_MERGE_NOSEQ = 0, OR_MERGE_GLOBAL = 1 };
#define OR_POOL_HALF 64      /* learned representatives: candidates per pool half */
#define OR_COVER_SAMPLE 4096 /* learned representatives: stride sample of the coverage count */

typedef struct {
    int32_t partitioning, p, m_per_dim[16], slice_dim;
    int32_t reps, n_reps, grid_filter, grid_filter_m;
    int32_t merge, threads;
    uint64_t seed;           /* Random partitioning and random representatives */
    const double *learned;   /* OR_REPS_LEARNED: the scorer's score of every point */
} or_opts;

typedef struct {
    int64_t n_in, n_after_grid, n_reps_kept, n_after_reps, size_u, size_sky, tests;
    int64_t tests_local, tests_merge;   /* the two parts of `tests` */
    int64_t n_reps;                     /* representatives chosen (before the self-filter) */
} or_stats;

typedef struct {
    const float *pts; int64_t n; int d; const double *sums;
    int32_t np; const int64_t *off; const int64_t *members;   /* CSR of alive points per partition */
    uint8_t *local;                                           /* by id: in u */
    int64_t *uorder;                                          /* u_i in SFS order, at off[i] */
    int64_t *local_sizes; int64_t *tests_per_part;
    /* merge */
    const int64_t *uoff; const int64_t *umem;                /* CSR of u per partition, SFS order */
    const uint8_t *pd;                                        /* np x np: pd[i*np+j] */
    uint8_t *out;                                             /* by id: in Sky */
    int64_t *merge_tests;
    atomic_long next;
} pipe_job;

static void *local_worker(void *arg)
{
    pipe_job *J = arg;
    for (;;) {
        long i = atomic_fetch_add(&J->next, 1);
        if (i >= J->np) break;
        int64_t t = 0;
        J->local_sizes[i] = sfs_subset(J->pts, J->n, J->d, J->sums, J->members + J->off[i],
                                       J->off[i + 1] - J->off[i], J->local, &t, J->uorder + J->off[i]);
        J->tests_per_part[i] = t;
    }
    return NULL;
}

/* NoSeq for the points of u_i: each is kept iff no point of pd_i dominates it. */
static void *merge_worker(void *arg)
{
    pipe_job *J = arg;
    sfs_ctx key = {J->pts, J->n, J->d, J->sums};
    for (;;) {
        long i = atomic_fetch_add(&J->next, 1);
        if (i >= J->np) break;
        int64_t t_cnt = 0;
        for (int64_t a = J->uoff[i]; a < J->uoff[i + 1]; ++a) {
            const int64_t t = J->umem[a];
            int dominated = 0;
            for (int32_t j = 0; j < J->np && !dominated; ++j) {
                if (!J->pd[(int64_t)i * J->np + j]) continue;
                for (int64_t b = J->uoff[j]; b < J->uoff[j + 1]; ++b) {
                    if (cmp_sfs(&J->umem[b], &t, &key) >= 0) break;   /* the rest come after t */
                    ++t_cnt;
                    if (dom_soa(J->pts, J->n, J->d, J->umem[b], t)) { dominated = 1; break; }
                }
            }
            J->out[t] = (uint8_t)!dominated;
        }
        J->merge_tests[i] = t_cnt;
    }
    return NULL;
}

static void run_workers(void *(*fn)(void *), pipe_job *J, int threads)
{
    atomic_store(&J->next, 0);
    if (threads <= 1) { fn(J); return; }
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)threads);
    for (int i = 0; i < threads; ++i) pthread_create(&th[i], NULL, fn, J);
    for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
    free(th);
}

/* Returns |Sky| >= 0, or a negative error: -1 bad options, -3 range.
 * rep_ids / rep_keep (nullable) receive the chosen representatives and their
 * self-filter flags (room for n_reps + p entries); rep_pool (nullable, 2 * 64
 * entries) the learned pool. */
int64_t or_pipeline(const float *pts, int64_t n, int32_t d, const or_opts *o, const float *scores,
                    uint8_t *in_sky, or_stats *st, int64_t *part_sizes, int64_t *part_kept,
                    int64_t *local_sizes, int64_t *rep_ids, uint8_t *rep_keep, int64_t *rep_pool)
{
    memset(st, 0, sizeof(*st));
    st->n_in = n;
    int np = o->p;
    if (o->partitioning == OR_PART_NONE) np = 1;
    if (np < 1 || d < 1 || d > 16) return -1;
    if (o->reps == OR_REPS_LEARNED && !o->learned) return -1;
    if (o->reps == OR_REPS_SCORES && !scores) return -1;
    int64_t N1 = n > 0 ? n : 1;
    uint8_t *alive = malloc((size_t)N1);
    for (int64_t i = 0; i < n; ++i) { alive[i] = 1; in_sky[i] = 0; }

    /* 1. Partition ids of all points. */
    uint32_t *part = calloc((size_t)N1, sizeof(uint32_t));
    int32_t rc = 0;
    if (o->partitioning == OR_PART_GRID) {
        int64_t prod = 1;
        for (int k = 0; k < d; ++k) prod *= o->m_per_dim[k];
        if (prod != np) rc = -1; else rc = or_grid_cells(pts, n, d, o->m_per_dim, part);
    } else if (o->partitioning == OR_PART_ANGULAR) {
        int64_t prod = 1;
        for (int k = 0; k < d - 1; ++k) prod *= o->m_per_dim[k];
        if (d < 2 || prod != np) rc = -1; else rc = or_angular_cells(pts, n, d, o->m_per_dim, part);
    } else if (o->partitioning == OR_PART_SLICED) {
        rc = or_sliced_cells(pts, n, d, o->slice_dim, np, part);
    } else if (o->partitioning == OR_PART_RANDOM) {
        rc = or_random_cells(n, np, o->seed, part);
    }
    if (rc != 0) { free(part); free(alive); return rc; }

    /* 2. Grid Filtering. */
    st->n_after_grid = n;
    if (o->grid_filter) {
        int32_t mg[16];
        for (int k = 0; k < d; ++k)
            mg[k] = (o->partitioning == OR_PART_GRID) ? o->m_per_dim[k] : o->grid_filter_m;
        uint8_t *pr = malloc((size_t)N1);
        int64_t kept = or_grid_filter(pts, n, d, mg, pr);
        if (kept < 0) { free(pr); free(part); free(alive); return kept; }
        for (int64_t i = 0; i < n; ++i) if (pr[i]) alive[i] = 0;
        st->n_after_grid = kept;
        free(pr);
    }

    /* 3. Representative Filtering. */
    st->n_after_reps = st->n_after_grid;
    if (o->reps != OR_REPS_NONE && o->n_reps > 0 && n > 0) {
        const int64_t cap = (int64_t)o->n_reps + np;
        float *sc = malloc(sizeof(float) * (size_t)N1);
        int64_t *ids = malloc(sizeof(int64_t) * (size_t)cap);
        uint8_t *keep = malloc((size_t)cap);
        int64_t k = 0;
        if (o->reps == OR_REPS_REGION) {
            if (or_region_scores(pts, n, d, sc) != 0) { free(sc); free(ids); free(keep); free(part); free(alive); return -3; }
        } else if (o->reps == OR_REPS_RANDOM) or_random_scores(n, o->seed, sc);
        else if (o->reps == OR_REPS_SCORES) memcpy(sc, scores, sizeof(float) * (size_t)n);
        else or_sum_scores(pts, n, d, sc);
        if (o->reps == OR_REPS_SORTED_PART) {
            k = or_sorted_part_reps(sc, n, part, np, o->n_reps, ids);
        } else if (o->reps == OR_REPS_LEARNED) {
            int64_t pool[2 * OR_POOL_HALF];
            or_learned_pool(sc, o->learned, n, OR_POOL_HALF, pool);
            if (rep_pool) memcpy(rep_pool, pool, sizeof pool);
            k = or_learned_mix(pts, n, d, pool, OR_POOL_HALF, o->n_reps, OR_COVER_SAMPLE, ids, NULL);
        } else {
            k = or_select_reps(sc, n, o->n_reps, ids);
        }
        st->n_reps = k;
        st->n_reps_kept = or_rep_selfilter(pts, n, d, ids, k, keep);
        for (int64_t a = 0; a < k; ++a) {
            if (rep_ids) rep_ids[a] = ids[a];
            if (rep_keep) rep_keep[a] = keep[a];
        }
        int64_t surv = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (!alive[i]) continue;
            for (int64_t a = 0; a < k; ++a)
                if (keep[a] && dom_soa(pts, n, d, ids[a], i)) { alive[i] = 0; break; }
            surv += alive[i];
        }
        st->n_after_reps = surv;
        free(sc); free(ids); free(keep);
    }

    int64_t *off = calloc((size_t)np + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (part_sizes) part_sizes[part[i]]++;
        if (alive[i]) off[part[i] + 1]++;
    }
    for (int j = 0; j < np; ++j) {
        if (part_kept) part_kept[j] = off[j + 1];
        off[j + 1] += off[j];
    }
    int64_t *members = malloc(sizeof(int64_t) * (size_t)(off[np] > 0 ? off[np] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)np);
    memcpy(fill, off, sizeof(int64_t) * (size_t)np);
    for (int64_t i = 0; i < n; ++i) if (alive[i]) members[fill[part[i]]++] = i;

    /* 4. Local skylines, parallel over partitions. */
    double *sums = malloc(sizeof(double) * (size_t)N1);
    for (int64_t i = 0; i < n; ++i) sums[i] = sum64(pts, n, d, i);
    uint8_t *local = calloc((size_t)N1, 1);
    int64_t *uorder = malloc(sizeof(int64_t) * (size_t)(off[np] > 0 ? off[np] : 1));
    int64_t *lsz = calloc((size_t)np, sizeof(int64_t));
    int64_t *tpp = calloc((size_t)np, sizeof(int64_t));
    int64_t *mt = calloc((size_t)np, sizeof(int64_t));
    pipe_job J;
    memset(&J, 0, sizeof(J));
    J.pts = pts; J.n = n; J.d = d; J.sums = sums; J.np = np; J.off = off; J.members = members;
    J.local = local; J.uorder = uorder; J.local_sizes = lsz; J.tests_per_part = tpp; J.merge_tests = mt;
    int threads = o->threads > 0 ? o->threads : 1;
    run_workers(local_worker, &J, threads);

    /* u as CSR per partition, each u_j in SFS order. */
    int64_t *uoff = calloc((size_t)np + 1, sizeof(int64_t));
    for (int j = 0; j < np; ++j) {
        uoff[j + 1] = uoff[j] + lsz[j];
        if (local_sizes) local_sizes[j] = lsz[j];
    }
    st->size_u = uoff[np];
    int64_t *umem = malloc(sizeof(int64_t) * (size_t)(uoff[np] > 0 ? uoff[np] : 1));
    for (int j = 0; j < np; ++j)
        memcpy(umem + uoff[j], uorder + off[j], sizeof(int64_t) * (size_t)lsz[j]);

    /* 5. Merge. */
    int64_t tests = 0;
    for (int j = 0; j < np; ++j) tests += tpp[j];
    st->tests_local = tests;
    if (np == 1) {
        for (int64_t a = 0; a < uoff[1]; ++a) in_sky[umem[a]] = 1;
    } else if (o->merge == OR_MERGE_GLOBAL) {
        int64_t t = 0;
        sfs_subset(pts, n, d, sums, umem, uoff[np], in_sky, &t, NULL);
        tests += t;
    } else {
        uint8_t *pd = calloc((size_t)np * (size_t)np, 1);
        int32_t ci[16], cj[16];
        for (int i = 0; i < np; ++i) {
            for (int j = 0; j < np; ++j) {
                if (i == j) continue;
                if (o->partitioning == OR_PART_SLICED) pd[i * np + j] = (j < i);
                else if (o->partitioning == OR_PART_ANGULAR || o->partitioning == OR_PART_RANDOM)
                    pd[i * np + j] = 1;   /* u minus u_i (Section 4.2) */
                else if (o->partitioning == OR_PART_GRID) {
                    cell_coords((uint64_t)i, d, o->m_per_dim, ci);
                    cell_coords((uint64_t)j, d, o->m_per_dim, cj);
                    int le = 1;
                    for (int k = 0; k < d; ++k) if (cj[k] > ci[k]) { le = 0; break; }
                    pd[i * np + j] = (uint8_t)le;
                }
            }
        }
        J.uoff = uoff; J.umem = umem; J.pd = pd; J.out = in_sky;
        run_workers(merge_worker, &J, threads);
        for (int j = 0; j < np; ++j) tests += mt[j];
        free(pd);
    }
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) cnt += in_sky[i];
    st->size_sky = cnt;
    st->tests = tests;
    st->tests_merge = tests - st->tests_local;
    free(alive); free(part); free(off); free(members); free(fill); free(sums); free(local); free(uorder);
    free(lsz); free(tpp); free(mt); free(uoff); free(umem);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* O7: the monotone MLP scorer g(x) = w3 . relu(W2 relu(W1 x + b1) + b2) + b3, */
/* evaluated in float64. Parameter layout (flat): W1 [h][d], b1 [h],           */
/* W2 [h][h] (row = output unit), b2 [h], w3 [h], b3 [1].                     */
/* round_mode 0: pure float64. round_mode 1: the inputs and the weight        */
/* matrices are rounded to bfloat16 (round to nearest even) and the first      */
/* hidden activation is rounded to bfloat16 after the ReLU, the points where   */
/* the GPU scorer rounds; rounding counts as the identity in the backward pass.*/
/* ------------------------------------------------------------------------ */
static double bf16_rne(double v)
{
    float f = (float)v;           /* the GPU holds these values as float32 first */
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return f;   /* inf/nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

int64_t or_mlp_nparams(int32_t d, int32_t h) { return (int64_t)h * d + h + (int64_t)h * h + h + h + 1; }

/* Forward for n points. g[i] output. If acts != NULL it receives z1 (h) and
 * z2 (h) per point, laid out [i][2h]. */
void or_mlp_forward(const double *P, int32_t d, int32_t h, const float *pts, int64_t n,
                    int32_t round_mode, double *g, double *acts)
{
    const double *W1 = P, *b1 = W1 + (int64_t)h * d, *W2 = b1 + h, *b2 = W2 + (int64_t)h * h,
                 *w3 = b2 + h, *b3 = w3 + h;
    double *a1 = malloc(sizeof(double) * (size_t)h), *a2 = malloc(sizeof(double) * (size_t)h);
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < h; ++j) {
            double z = 0.0;
            for (int k = 0; k < d; ++k) {
                double w = W1[j * d + k];
                if (round_mode) w = bf16_rne(w);
                double x = (double)PT(pts, n, k, i);
                if (round_mode) x = bf16_rne(x);
                z += w * x;
            }
            z += b1[j];
            if (acts) acts[i * 2 * h + j] = z;
            double r = z > 0.0 ? z : 0.0;
            a1[j] = round_mode ? bf16_rne(r) : r;
        }
        for (int j = 0; j < h; ++j) {
            double z = 0.0;
            for (int k = 0; k < h; ++k) {
                double w = W2[j * h + k];
                if (round_mode) w = bf16_rne(w);
                z += w * a1[k];
            }
            z += b2[j];
            if (acts) acts[i * 2 * h + h + j] = z;
            a2[j] = z > 0.0 ? z : 0.0;
        }
        double o = 0.0;
        for (int j = 0; j < h; ++j) {
            double w = w3[j];
            if (round_mode) w = bf16_rne(w);
            o += w * a2[j];
        }
        g[i] = o + b3[0];
    }
    free(a1); free(a2);
}

/* Loss L = mean_i (g(x_i) - y_i)^2 over the n points and its gradient with
 * respect to every parameter (same flat layout), by the chain rule. */
double or_mlp_loss_grad(const double *P, int32_t d, int32_t h, const float *pts, int64_t n,
                        const double *y, int32_t round_mode, double *grad)
{
    const double *W1 = P, *b1 = W1 + (int64_t)h * d, *W2 = b1 + h, *b2 = W2 + (int64_t)h * h,
                 *w3 = b2 + h;
    int64_t np_ = or_mlp_nparams(d, h);
    double *gW1 = grad, *gb1 = gW1 + (int64_t)h * d, *gW2 = gb1 + h, *gb2 = gW2 + (int64_t)h * h,
           *gw3 = gb2 + h, *gb3 = gw3 + h;
    for (int64_t q = 0; q < np_; ++q) grad[q] = 0.0;
    double *acts = malloc(sizeof(double) * 2 * (size_t)h * (size_t)(n > 0 ? n : 1));
    double *g = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    or_mlp_forward(P, d, h, pts, n, round_mode, g, acts);
    double *a1 = malloc(sizeof(double) * (size_t)h), *a2 = malloc(sizeof(double) * (size_t)h);
    double *dz2 = malloc(sizeof(double) * (size_t)h), *dz1 = malloc(sizeof(double) * (size_t)h);
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *z1 = acts + i * 2 * h, *z2 = z1 + h;
        double e = g[i] - y[i];
        loss += e * e;
        double dg = 2.0 * e / (double)n;
        for (int j = 0; j < h; ++j) {
            double r = z1[j] > 0.0 ? z1[j] : 0.0;
            a1[j] = round_mode ? bf16_rne(r) : r;
            a2[j] = z2[j] > 0.0 ? z2[j] : 0.0;
        }
        for (int j = 0; j < h; ++j) {
            double w = round_mode ? bf16_rne(w3[j]) : w3[j];
            gw3[j] += dg * a2[j];
            dz2[j] = (z2[j] > 0.0) ? dg * w : 0.0;
        }
        gb3[0] += dg;
        for (int k = 0; k < h; ++k) dz1[k] = 0.0;
        for (int j = 0; j < h; ++j) {
            gb2[j] += dz2[j];
            for (int k = 0; k < h; ++k) {
                double w = round_mode ? bf16_rne(W2[j * h + k]) : W2[j * h + k];
                gW2[j * h + k] += dz2[j] * a1[k];
                dz1[k] += w * dz2[j];
            }
        }
        for (int k = 0; k < h; ++k) {
            double dz = (z1[k] > 0.0) ? dz1[k] : 0.0;
            gb1[k] += dz;
            for (int c = 0; c < d; ++c) {
                double x = (double)PT(pts, n, c, i);
                if (round_mode) x = bf16_rne(x);
                gW1[k * d + c] += dz * x;
            }
        }
    }
    free(acts); free(g); free(a1); free(a2); free(dz2); free(dz1);
    return n > 0 ? loss / (double)n : 0.0;
}

/* One Adam step (Kingma & Ba) on the float64 parameters, then projection of
 * the weight matrices (not the biases) onto w >= 0, which keeps g monotone.
 * t is the 1-based step number. */
void or_mlp_adam(double *P, double *m, double *v, const double *grad, int32_t d, int32_t h,
                 double lr, double beta1, double beta2, double eps, int64_t t)
{
    int64_t np_ = or_mlp_nparams(d, h);
    int64_t nW1 = (int64_t)h * d, nW2 = (int64_t)h * h;
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t q = 0; q < np_; ++q) {
        m[q] = beta1 * m[q] + (1.0 - beta1) * grad[q];
        v[q] = beta2 * v[q] + (1.0 - beta2) * grad[q] * grad[q];
        double mh = m[q] / c1, vh = v[q] / c2;
        P[q] -= lr * mh / (sqrt(vh) + eps);
        int is_weight = (q < nW1) || (q >= nW1 + h && q < nW1 + h + nW2) ||
                        (q >= nW1 + h + nW2 + h && q < nW1 + h + nW2 + h + h);
        if (is_weight && P[q] < 0.0) P[q] = 0.0;
    }
}
