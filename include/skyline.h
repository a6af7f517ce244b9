/*
 * skyline.h -- C-ABI of the MI355X (gfx950) partitioned-skyline library.
 *
 * Paper: P. Ciaccia, D. Martinenghi, "Optimization Strategies for Parallel
 * Computation of Skylines", arXiv 2411.14968.
 *
 * The library computes the skyline (Def. 1, Section 2) of N points in d
 * dimensions with the paper's parallel pattern (Algorithm 2, Section 3):
 * partition (Grid, Section 3.2; Angular, Section 3.3 and Eq. (1); Sliced,
 * Section 3.4), prune (Grid Filtering, Section 3.2; Representative Filtering,
 * Section 4.1), compute local skylines with SFS semantics (Algorithm 1), and
 * merge them (NoSeq, Proposition 2 and Section 4.2, or the sequential final
 * round of Algorithm 2). A small monotone MLP scorer can replace the
 * coordinate sum for choosing representatives and for the presort order.
 *
 * Conventions shared by every entry point:
 *  - Points are float32 in SoA layout on the device: coordinate k of point i
 *    is pts[k * n + i]. 1 <= d <= 16, 0 <= n < 2^31.
 *  - Smaller is better in every dimension. The input is a multiset: exact
 *    duplicates never dominate each other. -0.0 is treated as +0.0.
 *  - NaN or infinite coordinates are rejected with SKY_ERR_NONFINITE.
 *  - Grid, Angular and Grid Filtering need coordinates in [0, 1]; a value
 *    outside gives SKY_ERR_RANGE.
 *  - Every function returns SKY_OK (0) or a negative error code; the message
 *    of the last error of a context is available from sky_last_error().
 *  - Device pointers are plain HIP device addresses; `stream` is a hipStream_t
 *    passed as void* (NULL = the default stream). The caller owns every
 *    pointer it passes; the library keeps none of them after a call returns.
 *  - A context owns all device workspace (it grows and is reused) and is not
 *    thread-safe: use one context per host thread.
 */
#ifndef SKYLINE_H
#define SKYLINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sky_ctx sky_ctx;
typedef struct sky_mlp sky_mlp;

enum {
    SKY_OK = 0,
    SKY_ERR_INVALID_ARG = -1,  /* bad size, option or pointer                     */
    SKY_ERR_NONFINITE = -2,    /* NaN or Inf coordinate                           */
    SKY_ERR_RANGE = -3,        /* coordinate outside [0,1] where the option needs it */
    SKY_ERR_CAPACITY = -4,     /* output buffer too small; *out_n = size needed   */
    SKY_ERR_OOM = -5,          /* device or pinned allocation failed              */
    SKY_ERR_HIP = -6,          /* a HIP runtime call failed                       */
    SKY_ERR_MODEL = -7,        /* learned option without a usable model           */
    SKY_ERR_IO = -8,           /* a file could not be read or written             */
    SKY_ERR_INTERNAL = -9      /* a self-check failed (e.g. results that differ)  */
};

/* Partitioning strategy (Section 3). NONE is a single partition. RANDOM
 * (Section 3.1) spreads the points at random over p equal-sized partitions:
 * point i goes to floor(r * p / n), r its rank in the order of
 * (floor(h_i / 2^32), i), h_i = SplitMix64 draw i from opts.seed (the output
 * for state seed + (i + 1) * 0x9E3779B97F4A7C15); its NoSeq candidates are all
 * other partitions (Section 4.2). */
enum { SKY_PART_NONE = 0, SKY_PART_GRID = 1, SKY_PART_ANGULAR = 2, SKY_PART_SLICED = 3, SKY_PART_RANDOM = 4 };
/* Representatives (Section 4.1). SORTED: the n_reps smallest by (float32
 * sequential coordinate sum, id). LEARNED (needs opts.model): a pool of the 64
 * smallest by sum and the 64 smallest by (MLP score, id), a learned one already
 * among the sum ones dropped. With R = min(n_reps, 64) and m_i = floor(i*R/4),
 * candidate set i (i = 0..4) is the first R - m_i sum points plus the first m_i
 * learned ones; the set that dominates the most points of a fixed stride
 * sample (input ids floor(s*N/M), s < M = min(N, 4096)) is used, ties to the
 * smaller i. Either kind only prunes with real points, so the skyline is
 * unchanged. */
/* REGION: the n_reps smallest by (-V, id), V = float32 product of (1 - x_k)
 * in coordinate order, the volume of the dominance region on [0,1]^d (needs
 * every coordinate in [0,1], else SKY_ERR_RANGE). RANDOM: a uniform sample,
 * the n_reps smallest by (floor(g_i / 2^40) * 2^-24, id), g_i = SplitMix64
 * draw i from opts.seed XOR 0xD1B54A32D192ED03. */
/* SORTED_PART: Sorted taken per partition (Section 4.1, the first tuples of
 * each partition after sorting): the kp = ceil(n_reps / p) smallest points of
 * every partition by (float32 sum, id), over all of its points, partition 0's
 * first; p * kp must not exceed 256. */
enum { SKY_REPS_NONE = 0, SKY_REPS_SORTED = 1, SKY_REPS_LEARNED = 2, SKY_REPS_REGION = 3, SKY_REPS_RANDOM = 4,
       SKY_REPS_SORTED_PART = 5 };
/* Merge of the local skylines: NoSeq (Proposition 2) or the final SFS round. */
enum { SKY_MERGE_NOSEQ = 0, SKY_MERGE_GLOBAL = 1 };
/* SFS presort order inside each partition (Algorithm 1 needs a topological
 * sort: any monotone score; points with equal scores are tested against each
 * other both ways). SUM: the coordinate sum. LEARNED: the learned score (needs
 * opts.model). ZORDER: the Z-order (Morton) code of coordinates quantised on
 * the input's bounding box, also monotone; it keeps nearby points together, so
 * whole blocks of a scan window can be skipped by their lower corner. The
 * skyline is the same under every order. */
/* ZORDER_SUM: the Z-order code with the coordinate sum below it as a second
 * key word (also monotone), so that points sharing a Z-order cell are ordered
 * by their sum and runs of equal keys stay short on data with many ties or a
 * skewed spread; it costs a sort key 32 bits wider. From d = 7, ZORDER sorts a
 * 64-bit key (7 to 9 bits per coordinate up to d = 9) rather than 24 or 32 bits,
 * where the code would keep only two or three bits per coordinate. */
enum { SKY_PRESORT_SUM = 0, SKY_PRESORT_LEARNED = 1, SKY_PRESORT_ZORDER = 2, SKY_PRESORT_ZORDER_SUM = 3 };

typedef struct sky_opts {
    int32_t partitioning;     /* SKY_PART_*                                           */
    int32_t p;                /* number of partitions (ignored for NONE)               */
    int32_t m_per_dim[16];    /* Grid: slices per dimension (d entries, product = p);  */
                              /* Angular: slices per angle (d-1 entries, product = p); */
                              /* all zero: derive m with m^d = p (Grid) or            */
                              /* m^(d-1) = p (Angular), error if p is not such a power */
    int32_t slice_dim;        /* Sliced: the dimension sorted on                       */
    int32_t reps;             /* SKY_REPS_*                                           */
    int32_t n_reps;           /* number of representatives selected, 1..256           */
    int32_t grid_filter;      /* 1: Grid Filtering on                                  */
    int32_t grid_filter_m;    /* slices per dimension of the filter grid when the      */
                              /* partitioning is not Grid (Grid uses its own cells);   */
                              /* m^d must be <= 65536                                  */
    int32_t merge;            /* SKY_MERGE_*                                          */
    int32_t presort;          /* SKY_PRESORT_*                                        */
    const sky_mlp *model;     /* scorer for the learned options, else NULL             */
    uint32_t flags;           /* SKY_FLAG_* bits, 0 by default                         */
    uint64_t seed;            /* random choices (RANDOM partitioning / reps), 0 default */
} sky_opts;

/* Counts of one sky_skyline call. Every count is a definition of a set, so it
 * does not depend on evaluation order. */
typedef struct sky_stats {
    int64_t n_in;             /* N                                                     */
    int64_t n_after_grid;     /* points not discarded by Grid Filtering                */
    int64_t n_reps_kept;      /* representatives left after their self-filter          */
    int64_t n_after_reps;     /* points surviving both filters                         */
    int64_t size_u;           /* size of the union of the local skylines               */
    int64_t size_sky;         /* size of the skyline                                   */
    int32_t n_parts;          /* partitions used                                       */
    int32_t reserved;
    const int64_t *part_sizes;  /* [n_parts] points per partition before filtering;    */
    const int64_t *part_kept;   /* [n_parts] points per partition after filtering;     */
    const int64_t *local_sizes; /* [n_parts] |u_i|; the three arrays are host memory   */
                                /* owned by the context, valid until its next call     */
    const int64_t *rep_ids;     /* [n_reps] chosen representative ids: Sorted in score  */
                                /* order; learned: the chosen set's sum part, then its  */
                                /* learned part, each in its list order                 */
    const uint8_t *rep_keep;    /* [n_reps] 1 if kept by the self-filter               */
    int32_t n_reps;
    int32_t n_pool;             /* learned representatives: pool size (else 0)         */
    const int64_t *rep_pool;    /* [n_pool] pool slot ids, -1 for an empty slot or a   */
                                /* learned candidate already among the sum candidates  */
    float ms_total;             /* device time of the call, milliseconds               */
    float ms_phase[8];          /* with SKY_FLAG_PHASE_TIMES: device time of each step, */
                                /* ms: 0 ingest, scores and the Sliced rank sort, 1     */
                                /* representative selection, 2 filters and partition    */
                                /* ids, 3 presort and chunking,                         */
                                /* 4 the local-skyline kernel alone, 5 union of the     */
                                /* local skylines, 6 the merge kernel alone (NoSeq) or  */
                                /* the final SFS round, 7 output                        */
    int64_t work[6];            /* with SKY_FLAG_COUNT_WORK: lane dominance tests issued */
                                /* by the dominance kernels (window records scanned x   */
                                /* the query slots of the wave, dead slots included):   */
                                /* 0 local-skyline kernel, 1 its block-corner checks,   */
                                /* 2 merge kernel (NoSeq or final round), 3 its corner  */
                                /* checks; 4, 5: the tests of 0 and 2 whose query point */
                                /* was still alive                                      */
    int64_t tests;              /* with SKY_FLAG_COUNT_WORK: dominance tests performed   */
                                /* for live query points, work[4] + work[5] (Section 2: */
                                /* a test is d coordinate compares); else 0             */
} sky_stats;

/* sky_opts.flags bits */
enum {
    SKY_FLAG_PHASE_TIMES = 1,   /* record one HIP event per step (small overhead)          */
    SKY_FLAG_COUNT_WORK = 2,    /* count the dominance kernels' work into sky_stats.work    */
    SKY_FLAG_NO_GRAPH = 4       /* launch every kernel of the call, never a captured graph  */
};

/* Create a context on HIP device `device`. */
int sky_create(sky_ctx **out, int32_t device);
void sky_destroy(sky_ctx *ctx);
/* Message of the last error on this context ("" if none). Owned by ctx. */
const char *sky_last_error(const sky_ctx *ctx);
/* Fill opts with defaults: Sliced on dimension 0, p = 16, 64 Sorted
 * representatives, NoSeq merge, Z-order presort, no Grid Filtering. */
void sky_opts_default(sky_opts *opts);

/*
 * Skyline of n points (Def. 1) through Algorithm 2 with the options in *opts.
 *   pts      device, float32 SoA (d, n), read only.
 *   out_ids  host memory, room for out_cap int64: receives the skyline as
 *            ascending, unique, 0-based point ids. out_cap = n always suffices.
 *   out_n    receives the skyline size (also on SKY_ERR_CAPACITY).
 *   stats    optional (NULL allowed).
 * Blocking: the call synchronises `stream` before returning, because the
 * result size is data dependent. The result does not depend on the options
 * (Propositions 1 and 2; representatives only remove dominated points).
 * A call with stats == NULL and no flags replays a HIP graph of its launch
 * sequence, captured on its first occurrence and kept in the context (up to 4,
 * keyed by the input pointer and size, the options, the learned model, the
 * output buffer, the work splits and the workspace; a workspace that grows
 * drops them). The model's weights are read when the graph runs, so training
 * between calls is seen. SKY_FLAG_NO_GRAPH launches the kernels one by one
 * instead.
 */
int sky_skyline(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const sky_opts *opts,
                int64_t *out_ids, int64_t out_cap, int64_t *out_n, sky_stats *stats,
                void *stream);

/* Batched skylines: n_inst independent instances in one launch sequence per
 * record width (the NoSeq method of Algorithm 2 with each instance as an outer
 * partition level). Instance i has ns[i] points of ds[i] coordinates, stored
 * as SoA (ds[i], ns[i]) float32 in device memory; the instances follow each
 * other in pts (instance i starts at float sum_{j<i} ds[j]*ns[j]). Options:
 * Sliced on dimension 0 with p <= 4096 slices per instance (or no
 * partitioning), Sorted representatives per instance (or none), NoSeq merge,
 * Z-order or sum presort; anything else is SKY_ERR_INVALID_ARG.
 *   out_ids   host, room for out_cap int64: instance after instance, each
 *             instance's skyline as ascending 0-based ids of its own points.
 *   out_offs  host, n_inst + 1 entries: instance i's ids are
 *             out_ids[out_offs[i] .. out_offs[i+1]). Filled also on
 *             SKY_ERR_CAPACITY (out_offs[n_inst] is the size needed).
 *   bstats    optional (NULL allowed).
 * Blocking, like sky_skyline. Instances with fewer coordinates than others of
 * the same record width get zero coordinates, which changes no result. */
typedef struct sky_batch_stats {
    int64_t n_total;   /* points over all instances                      */
    int64_t size_sky;  /* skyline points over all instances              */
    int32_t n_groups;  /* launch sequences (one per record width)        */
    float ms_total;    /* device time of the sequences, milliseconds     */
} sky_batch_stats;

int sky_skyline_batch(sky_ctx *ctx, const float *pts, const int64_t *ns, const int32_t *ds, int32_t n_inst,
                      const sky_opts *opts, int64_t *out_ids, int64_t out_cap, int64_t *out_offs,
                      sky_batch_stats *bstats, void *stream);

/* ---------------------------------------------------------------------------
 * Work splits of the dominance kernels (the local-skyline kernel, which also
 * runs the final round, and the NoSeq merge kernel). They change the time of a
 * call, never its result: every split runs the same dominance tests on the
 * same candidate sets (Algorithm 1 inside Algorithm 2, Proposition 2).
 * The context holds a tuning table with one entry per (record width
 * DP = roundup(d + 2, 4), floor(log2 n)); a call with no entry uses the
 * built-in splits (sky_tune_default). Batched calls look up each launch
 * sequence by its record width and its total point count.
 * ------------------------------------------------------------------------- */
typedef struct sky_tune_params {
    int32_t local_ppl;   /* query points per lane of the local kernel: 1, 2 or 4 (a query group is 64 * ppl points) */
    int32_t local_seg;   /* smallest window segment of a local item, records: a power of two in [256, 8192]      */
    int32_t merge_ppl;   /* query points per lane of the merge kernel: 1, 2 or 4                                  */
    int32_t merge_seg;   /* window segment of a merge item, records: a power of two in [256, 8192]               */
    int32_t wg_per_cu;   /* persistent workgroups of 4 waves per compute unit: 1 .. 8                             */
} sky_tune_params;

/* The built-in splits for d coordinates. */
void sky_tune_default(int32_t d, sky_tune_params *out);
/* Set the table entry that calls with d coordinates and n points use.
 * SKY_ERR_INVALID_ARG for a field outside its range, d outside [1, 16] or n < 1. */
int sky_tune_set(sky_ctx *ctx, int32_t d, int64_t n, const sky_tune_params *params);
/* The splits a call with d coordinates and n points would use. Returns 1 when
 * they come from the table, 0 for the built-in ones, < 0 on an error. */
int sky_tune_get(const sky_ctx *ctx, int32_t d, int64_t n, sky_tune_params *out);
/* Drop every table entry. */
void sky_tune_clear(sky_ctx *ctx);
/* Save the table as text: a header line "skyline-tune 1 <arch> <compute units>",
 * then one line per entry "<DP> <log2 n> <local_ppl> <local_seg> <merge_ppl>
 * <merge_seg> <wg_per_cu>". SKY_ERR_IO when the file cannot be written. */
int sky_tune_save(const sky_ctx *ctx, const char *path);
/* Load a saved table into the context (entries replace those with the same
 * key). SKY_ERR_IO when the file cannot be read; SKY_ERR_INVALID_ARG when it is
 * malformed or was tuned on another architecture or compute-unit count (the
 * context's table is then unchanged). */
int sky_tune_load(sky_ctx *ctx, const char *path);

/* Autotune the splits for one input: time sky_skyline(pts, n, d, opts) under
 * candidate splits by coordinate descent over the five fields (two passes,
 * starting from the current entry), each candidate by the median device time
 * of `trials` calls after one untimed call, and store the fastest in the table
 * entry of (d, n). Every candidate's ids must equal the first call's, else
 * SKY_ERR_INTERNAL. best (nullable) receives the chosen splits, best_ms and
 * base_ms (nullable) its median time and that of the starting splits.
 * Arguments as in sky_skyline; trials in [1, 50]. */
int sky_autotune(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const sky_opts *opts, int32_t trials,
                 sky_tune_params *best, float *best_ms, float *base_ms, void *stream);
/* The same for a batch: the candidates are applied to the table entry of
 * every launch sequence of the batch, timed by sky_batch_stats.ms_total, and
 * the fastest is stored for all of them. Arguments as in sky_skyline_batch. */
int sky_autotune_batch(sky_ctx *ctx, const float *pts, const int64_t *ns, const int32_t *ds, int32_t n_inst,
                       const sky_opts *opts, int32_t trials, sky_tune_params *best, float *best_ms, float *base_ms,
                       void *stream);

/* ---------------------------------------------------------------------------
 * Learned scorer g(x) = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with all weight
 * matrices >= 0, hence monotone non-decreasing in every coordinate, so sorting
 * by g is a topological sort with respect to dominance (Section 2, Algorithm 1).
 * It generalises the dominance-region volume score of Section 4.1.
 * Parameters, flat float32, in this order: W1 [h][d], b1 [h], W2 [h][h]
 * (row = output unit), b2 [h], w3 [h], b3 [1]; h*d + h*h + 3h + 1 values.
 * The context keeps float32 master weights; scoring uses bfloat16 copies of the
 * weight matrices (round to nearest even) with float32 accumulation, and rounds
 * the first hidden activation to bfloat16.
 * ------------------------------------------------------------------------- */
int64_t sky_mlp_nparams(int32_t d, int32_t hidden);
/* init: host, nparams floats, or NULL for a seeded default initialisation.
 * Negative weight-matrix entries are projected to 0. hidden must be 64. */
int sky_mlp_create(sky_ctx *ctx, int32_t d, int32_t hidden, const float *init, uint64_t seed,
                   sky_mlp **out);
void sky_mlp_destroy(sky_mlp *model);
/* Copy the float32 master parameters to host memory (cap >= nparams). */
int sky_mlp_get_params(const sky_mlp *model, float *host_out, int64_t cap);
/* Save / load the parameters and optimiser state (little-endian binary file). */
int sky_mlp_save(const sky_mlp *model, const char *path);
int sky_mlp_load(sky_ctx *ctx, const char *path, sky_mlp **out);
/* Scores of n points: out device float32[n]. */
int sky_mlp_score(sky_ctx *ctx, const sky_mlp *model, const float *pts, int64_t n, int32_t d,
                  float *out, void *stream);
/* Mean squared error of g against targets y (device float32[n]) over the n
 * points and its gradient: grad device float32[nparams], loss device float32[1].
 * The bfloat16 roundings of the forward pass count as the identity. */
int sky_mlp_loss_grad(sky_ctx *ctx, const sky_mlp *model, const float *pts, int64_t n, int32_t d,
                      const float *y, float *grad, float *loss, void *stream);
/* One Adam step on the master weights with gradient grad (device), then the
 * projection of the weight matrices onto >= 0 and the bfloat16 refresh.
 * step is 1-based. */
int sky_mlp_adam_step(sky_ctx *ctx, sky_mlp *model, const float *grad, float lr, float beta1,
                      float beta2, float eps, int64_t step, void *stream);

typedef struct sky_train_opts {
    int32_t epochs;           /* passes over the data                                  */
    int32_t batch;            /* mini-batch size                                       */
    float lr, beta1, beta2, eps;
} sky_train_opts;

/* Train on n points with targets y (device float32[n]); mini-batches are the
 * consecutive slices of the given order (shuffle before calling). loss_out
 * (host, nullable) receives the mean loss of the last epoch. */
int sky_mlp_train(sky_ctx *ctx, sky_mlp *model, const float *pts, int64_t n, int32_t d,
                  const float *y, const sky_train_opts *topts, float *loss_out, void *stream);

/* Dominance counts (Def. 2): out[i] = #{ j in sample : point i dominates
 * point sample[j] }. sample: device uint32[m] point ids; out: device uint32[n]. */
int sky_domcount(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *sample,
                 int64_t m, uint32_t *out, void *stream);
/* The reverse count (Def. 2 read the other way): out[i] = #{ j in by : point
 * by[j] dominates point i }, e.g. whether a set of representatives (Section 4.1)
 * prunes point i. by: device uint32[m] point ids; out: device uint32[n]. */
int sky_domby(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *by, int64_t m,
              uint32_t *out, void *stream);

/* Training targets of the scorer from the method's own dominance test in
 * count mode (Def. 2). The residual sample keeps the points sample[j] that no
 * point reps[r] dominates (with reps the input's own Sorted representatives,
 * Section 4.1, what they prune is left out); dc(i) counts the residual points
 * that point i dominates, and
 *     y[i] = -log1p(dc(i) * n / m) / log1p(n)
 * in float64, rounded once to float32: 0 for a point that dominates nothing,
 * -1 for one that dominates all m sample points (m is the full sample's size).
 *   sample: device uint32[m] point ids; reps: device uint32[nreps] point ids
 *   (NULL when nreps = 0); y: device float32[n]; kept_out (host, nullable):
 *   the residual sample's size. Blocking. Ids must be < n. */
int sky_mlp_targets(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *sample, int64_t m,
                    const uint32_t *reps, int64_t nreps, float *y, int64_t *kept_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the targets
 * of sky_mlp_targets, computed by the same kernels, with the residual sample in
 * a library-owned static device array of SKY_NOALLOC_MAX_M ids (4 MiB per
 * device, held until the process ends; its address is looked up per device by
 * sky_create) instead of an allocation. Allocates nothing, does not
 * synchronise and issues no memset, so it can be captured into a graph.
 *   kept_dev: device uint32[1] receiving the residual sample's size, or NULL.
 * m > SKY_NOALLOC_MAX_M gives SKY_ERR_CAPACITY. Every call on a device shares
 * that device's array: calls that overlap on one device (other streams, other
 * host threads, other contexts) race and must be serialised by the caller. */
#define SKY_NOALLOC_MAX_M (1u << 20)
int sky_mlp_targets_noalloc(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *sample,
                            int64_t m, const uint32_t *reps, int64_t nreps, float *y, uint32_t *kept_dev,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SKYLINE_H */
