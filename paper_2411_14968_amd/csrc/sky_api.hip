// C-ABI of the skyline library: context, workspace and the launch sequence of
// one skyline call (Algorithm 2 with the options of Sections 3 and 4).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/skyline.h"
#include "sky_internal.h"
#include "sky_mlp.h"

__global__ void k_set_u32(uint32_t *p, uint32_t v) { *p = v; }

// ------------------------------------------------------------------ context
// Everything a captured sky_skyline launch sequence bakes in: the input, the
// options, the output destination, the work splits and the workspace
// generation (any reallocation makes older graphs unusable).
struct GraphKey {
    const float *pts;
    uint32_t n;
    int d, kind, p, slice_dim, reps, n_reps, gf, gf_m, merge, presort;
    uint64_t seed, model;   // model: the learned scorer's serial (0: none)
    int m[SKY_MAXD];
    int64_t *dst;
    uint32_t dcap;
    uint64_t gen;
    TuneParams tp;
    bool operator==(const GraphKey &o) const
    {
        return pts == o.pts && n == o.n && d == o.d && kind == o.kind && p == o.p && slice_dim == o.slice_dim &&
               reps == o.reps && n_reps == o.n_reps && gf == o.gf && gf_m == o.gf_m && merge == o.merge &&
               presort == o.presort && seed == o.seed && model == o.model && memcmp(m, o.m, sizeof m) == 0 &&
               dst == o.dst &&
               dcap == o.dcap &&
               gen == o.gen && tp.lppl == o.tp.lppl && tp.lseg == o.tp.lseg && tp.mppl == o.tp.mppl &&
               tp.mseg == o.tp.mseg && tp.wgcu == o.tp.wgcu;
    }
};
#define SKY_MAX_GRAPHS 4

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct sky_ctx {
    int device = 0;
    int n_cu = 256;
    std::string err;
    // device workspace
    DevBuf ctrl, score, score2, part, alive, occ, gdom, selhist, cand, rep_ids, rep_keep, krec, part_hist;
    DevBuf kA, kB, vA, vB, shist, wgcnt;
    DevBuf rec, wpos, sid, skey, in_u, poff, poff2, nch, st_off, scratch;
    DevBuf urec, uid, ukey, upoff, lsizes, skybits, udead, bmin, ubmin, zq, tick, wcnt, cover;
    DevBuf bpts, binst, bkrec, bmeta;   // batched skylines
    DevBuf qsel;                        // Sliced boundary selection: state, then the boundary keys
    // pinned host
    uint32_t *ctrl_h = nullptr;
    int64_t *ids_h = nullptr;
    size_t ids_h_cap = 0;
    int64_t *lsizes_h = nullptr;
    uint32_t *poff_h = nullptr;
    uint32_t *phist_h = nullptr;
    uint32_t *repids_h = nullptr;
    uint8_t *repkeep_h = nullptr;
    uint64_t *wcnt_h = nullptr;
    char *bmeta_h = nullptr;
    size_t bmeta_h_cap = 0;
    size_t np_cap = 0;
    // stats arrays handed out through sky_stats
    std::vector<int64_t> st_part_sizes, st_part_kept, st_local, st_rep_ids, st_rep_pool;
    std::vector<uint8_t> st_rep_keep;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_tie = nullptr;
    // a second stream (default priority) for work independent of the caller's
    // stream until a join: the Sliced boundary selection
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_mlp = nullptr;
    // captured launch sequences of sky_skyline (see GraphKey)
    hipStream_t cap = nullptr;   // capture happens here: the caller's stream may be the null stream
    uint64_t gen = 0;            // bumped whenever a workspace buffer moves
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
    hipEvent_t evp[9] = {};
    // tuning table: work splits of the dominance kernels per (record width
    // DP = 4 (row + 1), n in [2^b, 2^(b+1)))
    TuneParams tune[5][33] = {};
    bool tune_has[5][33] = {};
    std::string arch;   // device architecture name, the tuning table's scope
};

static bool tune_slot(int dp, uint64_t n, int *row, int *col)
{
    *row = dp / 4 - 1;
    *col = n ? 63 - __builtin_clzll(n) : 0;
    return *row >= 0 && *row < 5 && *col < 33;
}

static TuneParams tune_for(const sky_ctx *c, int d, uint64_t n)
{
    int r, b;
    if (tune_slot(sky_dp(d), n, &r, &b) && c->tune_has[r][b]) return c->tune[r][b];
    return tune_builtin(d);
}

static int set_err(sky_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIP_OK(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return set_err(ctx, SKY_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

static void drop_graphs(sky_ctx *ctx)
{
    ++ctx->gen;
    for (auto &g : ctx->graphs) hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
}

static int ensure(sky_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (b.bytes >= bytes) return SKY_OK;
    drop_graphs(ctx);
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        return set_err(ctx, SKY_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    }
    b.bytes = bytes;
    return SKY_OK;
}

template <typename T> static T *P(DevBuf &b) { return reinterpret_cast<T *>(b.p); }

extern "C" int sky_create(sky_ctx **out, int32_t device)
{
    if (!out) return SKY_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SKY_ERR_INVALID_ARG;
    sky_ctx *c = new sky_ctx();
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete c; return SKY_ERR_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        if (prop.multiProcessorCount > 0) c->n_cu = prop.multiProcessorCount;
        c->arch = prop.gcnArchName;
        const size_t colon = c->arch.find(':');   // drop feature suffixes such as ":sramecc+:xnack-"
        if (colon != std::string::npos) c->arch.resize(colon);
    }
    if (hipHostMalloc((void **)&c->ctrl_h, C_NUM * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SKY_ERR_OOM;
    }
    hipEventCreate(&c->ev0);
    hipEventCreate(&c->ev1);
    hipEventCreateWithFlags(&c->ev_tie, hipEventDisableTiming);
    hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    hipEventCreateWithFlags(&c->ev_mlp, hipEventDisableTiming);
    for (auto &e : c->evp) hipEventCreate(&e);
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        sky_destroy(c);
        return SKY_ERR_HIP;
    }
    if (device >= SKY_MAX_DEVICES || sky_noalloc_setup(device) != SKY_OK) {   // allocation-free entry point
        sky_destroy(c);
        return SKY_ERR_HIP;
    }
    *out = c;
    return SKY_OK;
}

extern "C" void sky_destroy(sky_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    DevBuf *bufs[] = {&c->ctrl, &c->score, &c->score2, &c->part, &c->alive, &c->occ, &c->gdom, &c->selhist,
                      &c->cand, &c->rep_ids, &c->rep_keep, &c->krec, &c->part_hist, &c->kA, &c->kB, &c->vA,
                      &c->vB, &c->shist, &c->wgcnt, &c->rec, &c->wpos, &c->sid, &c->skey, &c->in_u,
                      &c->poff, &c->poff2, &c->nch, &c->st_off, &c->scratch, &c->urec,
                      &c->uid, &c->ukey, &c->upoff, &c->lsizes, &c->skybits, &c->udead,
                      &c->bmin, &c->ubmin, &c->zq, &c->tick, &c->wcnt, &c->cover,
                      &c->bpts, &c->binst, &c->bkrec, &c->bmeta, &c->qsel};
    for (DevBuf *b : bufs)
        if (b->p) hipFree(b->p);
    if (c->ctrl_h) hipHostFree(c->ctrl_h);
    if (c->ids_h) hipHostFree(c->ids_h);
    if (c->lsizes_h) hipHostFree(c->lsizes_h);
    if (c->poff_h) hipHostFree(c->poff_h);
    if (c->phist_h) hipHostFree(c->phist_h);
    if (c->repids_h) hipHostFree(c->repids_h);
    if (c->repkeep_h) hipHostFree(c->repkeep_h);
    if (c->wcnt_h) hipHostFree(c->wcnt_h);
    if (c->bmeta_h) hipHostFree(c->bmeta_h);
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    if (c->ev_tie) hipEventDestroy(c->ev_tie);
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_join) hipEventDestroy(c->ev_join);
    if (c->ev_mlp) hipEventDestroy(c->ev_mlp);
    if (c->side) hipStreamDestroy(c->side);
    for (auto &g : c->graphs) hipGraphExecDestroy(g.second);
    if (c->cap) hipStreamDestroy(c->cap);
    for (auto &e : c->evp)
        if (e) hipEventDestroy(e);
    delete c;
}

extern "C" const char *sky_last_error(const sky_ctx *c) { return c ? c->err.c_str() : "null context"; }

int sky_ctx_device(const sky_ctx *c) { return c ? c->device : 0; }

extern "C" void sky_opts_default(sky_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->partitioning = SKY_PART_SLICED;
    o->p = 16;
    o->slice_dim = 0;
    o->reps = SKY_REPS_SORTED;
    o->n_reps = 64;
    o->grid_filter = 0;
    o->grid_filter_m = 0;
    o->merge = SKY_MERGE_NOSEQ;
    o->presort = SKY_PRESORT_ZORDER;
    o->model = nullptr;
}

// Integer m with m^e == p, or 0.
static int int_root(int p, int e)
{
    if (e <= 0) return p == 1 ? 1 : 0;
    for (int m = 1; m <= p; ++m) {
        long long v = 1;
        for (int i = 0; i < e && v <= p; ++i) v *= m;
        if (v == p) return m;
        if (v > p) break;
    }
    return 0;
}

static int bits_for(uint32_t v)   // ceil(log2(v)), v >= 1
{
    int b = 0;
    while ((1ull << b) < v) ++b;
    return b;
}

static int grow_pinned(sky_ctx *ctx, size_t np, size_t n_ids)
{
    if (np + 1 > ctx->np_cap) {
        if (ctx->lsizes_h) hipHostFree(ctx->lsizes_h);
        if (ctx->poff_h) hipHostFree(ctx->poff_h);
        if (ctx->phist_h) hipHostFree(ctx->phist_h);
        ctx->lsizes_h = nullptr; ctx->poff_h = nullptr; ctx->phist_h = nullptr;
        const size_t cap = np + 1;
        if (hipHostMalloc((void **)&ctx->lsizes_h, cap * sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&ctx->poff_h, cap * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&ctx->phist_h, cap * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
            ctx->np_cap = 0;
            return set_err(ctx, SKY_ERR_OOM, "pinned allocation failed");
        }
        ctx->np_cap = cap;
    }
    if (!ctx->repids_h) {
        if (hipHostMalloc((void **)&ctx->repids_h, (SKY_MAXREPS + 2 * SKY_POOL_HALF) * sizeof(uint32_t),
                          hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&ctx->repkeep_h, SKY_MAXREPS, hipHostMallocDefault) != hipSuccess)
            return set_err(ctx, SKY_ERR_OOM, "pinned allocation failed");
    }
    if (n_ids > ctx->ids_h_cap) {
        drop_graphs(ctx);
        if (ctx->ids_h) hipHostFree(ctx->ids_h);
        ctx->ids_h = nullptr;
        ctx->ids_h_cap = 0;
        if (hipHostMalloc((void **)&ctx->ids_h, n_ids * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
            return set_err(ctx, SKY_ERR_OOM, "pinned allocation failed");
        ctx->ids_h_cap = n_ids;
    }
    return SKY_OK;
}

// ------------------------------------------------------------------ skyline
extern "C" int sky_skyline(sky_ctx *ctx, const float *pts, int64_t n64, int32_t d, const sky_opts *opts,
                           int64_t *out_ids, int64_t out_cap, int64_t *out_n, sky_stats *stats, void *stream)
{
    if (!ctx) return SKY_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!opts || !out_n) return set_err(ctx, SKY_ERR_INVALID_ARG, "opts and out_n are required");
    *out_n = 0;
    if (d < 1 || d > SKY_MAXD) return set_err(ctx, SKY_ERR_INVALID_ARG, "d must be in [1, 16], got %d", d);
    if (n64 < 0 || n64 >= (1ll << 31)) return set_err(ctx, SKY_ERR_INVALID_ARG, "n must be in [0, 2^31)");
    if (n64 > 0 && !pts) return set_err(ctx, SKY_ERR_INVALID_ARG, "pts is NULL");
    if (out_cap > 0 && !out_ids) return set_err(ctx, SKY_ERR_INVALID_ARG, "out_ids is NULL");
    const uint32_t n = (uint32_t)n64;
    const sky_opts &o = *opts;
    int kind = o.partitioning;
    if (kind < SKY_PART_NONE || kind > SKY_PART_RANDOM)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "unknown partitioning %d", kind);
    int np = kind == SKY_PART_NONE ? 1 : o.p;
    if (np < 1 || np > SKY_MAX_GRID_CELLS) return set_err(ctx, SKY_ERR_INVALID_ARG, "p must be in [1, 65536]");
    if (o.reps < SKY_REPS_NONE || o.reps > SKY_REPS_SORTED_PART)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "unknown reps %d", o.reps);
    if (o.reps != SKY_REPS_NONE && (o.n_reps < 1 || o.n_reps > SKY_MAXREPS))
        return set_err(ctx, SKY_ERR_INVALID_ARG, "n_reps must be in [1, 256]");
    const int kp_part = o.reps == SKY_REPS_SORTED_PART ? (o.n_reps + np - 1) / np : 0;   // per partition
    if (o.reps == SKY_REPS_SORTED_PART && (int64_t)kp_part * np > SKY_MAXREPS)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "per-partition representatives: p * ceil(n_reps / p) exceeds 256");
    if (o.merge != SKY_MERGE_NOSEQ && o.merge != SKY_MERGE_GLOBAL)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "unknown merge %d", o.merge);
    if (o.presort != SKY_PRESORT_SUM && o.presort != SKY_PRESORT_LEARNED && o.presort != SKY_PRESORT_ZORDER &&
        o.presort != SKY_PRESORT_ZORDER_SUM)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "unknown presort %d", o.presort);
    const bool learned = o.reps == SKY_REPS_LEARNED || o.presort == SKY_PRESORT_LEARNED;
    if (learned) {
        if (!o.model) return set_err(ctx, SKY_ERR_MODEL, "learned option without a model");
        if (sky_mlp_dim(o.model) != d)
            return set_err(ctx, SKY_ERR_MODEL, "model is for d=%d, points have d=%d", sky_mlp_dim(o.model), d);
    }
    GridSpec pg{};
    pg.d = d;
    AngSpec ag{};
    ag.d = d;
    if (kind == SKY_PART_GRID) {
        bool given = false;
        for (int k = 0; k < d; ++k) given |= o.m_per_dim[k] != 0;
        long long prod = 1;
        for (int k = 0; k < d; ++k) {
            int m = given ? o.m_per_dim[k] : int_root(np, d);
            if (m < 1) return set_err(ctx, SKY_ERR_INVALID_ARG, "Grid: p=%d is not m^d and m_per_dim is unset", np);
            pg.m[k] = m;
            prod *= m;
        }
        if (prod != np) return set_err(ctx, SKY_ERR_INVALID_ARG, "Grid: product of m_per_dim (%lld) != p (%d)", prod, np);
    } else if (kind == SKY_PART_ANGULAR) {
        if (d < 2) {
            if (np != 1) return set_err(ctx, SKY_ERR_INVALID_ARG, "Angular needs d >= 2 for p > 1");
        } else {
            bool given = false;
            for (int k = 0; k < d - 1; ++k) given |= o.m_per_dim[k] != 0;
            long long prod = 1;
            for (int a = 0; a < d - 1; ++a) {
                int m = given ? o.m_per_dim[a] : int_root(np, d - 1);
                if (m < 1 || m > SKY_MAX_ANG_M)
                    return set_err(ctx, SKY_ERR_INVALID_ARG, "Angular: slices per angle must be in [1, 16] with product p");
                ag.m[a] = m;
                prod *= m;
                for (int k = 1; k < m; ++k) {
                    const double ang = (double)k * M_PI / (2.0 * (double)m);
                    const double tv = tan(ang);
                    ag.T[a][k] = tv * tv;
                }
            }
            if (prod != np) return set_err(ctx, SKY_ERR_INVALID_ARG, "Angular: product of slices (%lld) != p (%d)", prod, np);
        }
    } else if (kind == SKY_PART_SLICED) {
        if (o.slice_dim < 0 || o.slice_dim >= d) return set_err(ctx, SKY_ERR_INVALID_ARG, "slice_dim out of range");
    }
    GridSpec gg{};
    gg.d = d;
    const bool gf = o.grid_filter != 0;
    if (gf) {
        long long prod = 1;
        for (int k = 0; k < d; ++k) {
            const int m = kind == SKY_PART_GRID ? pg.m[k] : o.grid_filter_m;
            if (m < 1) return set_err(ctx, SKY_ERR_INVALID_ARG, "grid_filter_m must be >= 1");
            gg.m[k] = m;
            prod *= m;
            if (prod > SKY_MAX_GRID_CELLS)
                return set_err(ctx, SKY_ERR_INVALID_ARG, "Grid Filtering grid has more than 65536 cells");
        }
    }
    const bool need_range = gf || kind == SKY_PART_GRID || kind == SKY_PART_ANGULAR || o.reps == SKY_REPS_REGION;
    const bool own_scores = o.reps == SKY_REPS_REGION || o.reps == SKY_REPS_RANDOM;   // into score2

    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, SKY_ERR_HIP, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->n_in = n64;
        stats->n_parts = np;
    }
    if (n == 0) return SKY_OK;

    // ---------------------------------------------------------------- workspace
    const int DP = sky_dp(d);
    const TuneParams tp = tune_for(ctx, d, n);
    const int B = 64 * tp.lppl;
    const uint32_t max_chunks = n / (uint32_t)(LS_MIN_CHUNK) + (uint32_t)np + 2;
    const int G = sort_groups(n);
    int rc;
#define ENS(b, bytes) if ((rc = ensure(ctx, ctx->b, (bytes))) != SKY_OK) return rc
    ENS(ctrl, C_NUM * 4);
    ENS(score, (size_t)n * 4);
    if (learned || own_scores) ENS(score2, (size_t)n * 4);
    ENS(part, (size_t)n * 4);
    ENS(alive, (size_t)n);
    ENS(occ, SKY_MAX_GRID_CELLS / 8);
    ENS(gdom, SKY_MAX_GRID_CELLS / 8);
    ENS(selhist, SKY_SEL_WORDS * 4);
    ENS(cand, 3 * SKY_MAXREPS * 8);   // two selections, then the picks
    ENS(cover, (size_t)(2 * SKY_POOL_HALF) * 4);   // the learned pool's ids
    ENS(rep_ids, SKY_MAXREPS * 4);
    ENS(rep_keep, SKY_MAXREPS);
    ENS(krec, SKY_MAXREPS * 20 * 4);
    ENS(part_hist, (size_t)(np + 1) * 4);
    ENS(kA, (size_t)n * 8);
    ENS(kB, (size_t)n * 8);
    ENS(vA, (size_t)n * 4);
    ENS(vB, (size_t)n * 4);
    ENS(shist, ((size_t)256 * 1024 + 1024 + 64) * 4);
    ENS(wgcnt, (size_t)(n / 4096 + 8192 + 4200) * 4);
    ENS(rec, (size_t)n * DP * 4);
    ENS(wpos, (size_t)n * 4);
    ENS(sid, (size_t)n * 4);
    ENS(skey, (size_t)n * 8);
    ENS(in_u, (size_t)n + 512);   // dead flags; a group's tail may read past n
    ENS(poff, (size_t)(np + 2) * 4);
    ENS(poff2, 16);
    ENS(nch, (size_t)(np + 1) * 4);
    ENS(st_off, (size_t)(np + 2) * 4);
    ENS(scratch, ((size_t)2 * max_chunks + np + 8) * 4);
    ENS(urec, (size_t)n * DP * 4);
    ENS(uid, (size_t)n * 4);
    ENS(ukey, (size_t)n * 8);
    ENS(upoff, (size_t)(np + 2) * 4);
    ENS(lsizes, (size_t)(np + 1) * 8);
    ENS(skybits, ((size_t)n / 32 + 1) * 4);
    ENS(udead, (size_t)n + 512);
    // block corners (4 blocks past the last one are read, and ignored, by the batched scan), then
    // super-block corners
    ENS(bmin, sky_corner_words(n, DP) * 4);
    ENS(ubmin, sky_corner_words(n, DP) * 4);
    ENS(zq, (size_t)(2 * 16 * SKY_INGEST_MAX_WG + 64) * 4);
    ENS(tick, (size_t)3 * SKY_TICK_SET * 4);   // ticket counters: local, merge, final round
    ENS(qsel, (size_t)(SKY_QSEL_WORDS + SKY_QSEL_MAX_P) * 4);
    const bool count_work = (o.flags & SKY_FLAG_COUNT_WORK) != 0;
    if (count_work) {
        ENS(wcnt, (size_t)2 * SKY_TICK_C * 8 * 8);
        if (!ctx->wcnt_h && hipHostMalloc((void **)&ctx->wcnt_h, (size_t)2 * SKY_TICK_C * 8 * 8) != hipSuccess)
            return set_err(ctx, SKY_ERR_OOM, "pinned host allocation failed");
    }
    uint64_t *wcnt_l = count_work ? P<uint64_t>(ctx->wcnt) : nullptr;
    uint64_t *wcnt_m = count_work ? wcnt_l + SKY_TICK_C * 8 : nullptr;
#undef ENS
    if ((rc = grow_pinned(ctx, (size_t)np, (size_t)n)) != SKY_OK) return rc;

    uint32_t *ctrl = P<uint32_t>(ctx->ctrl);
    SortBufs sb{P<uint64_t>(ctx->kA), P<uint64_t>(ctx->kB), P<uint32_t>(ctx->vA), P<uint32_t>(ctx->vB),
                P<uint32_t>(ctx->shist), P<uint32_t>(ctx->shist) + 256 * 1024,
                P<uint32_t>(ctx->shist) + 256 * 1024 + 1024, G};
    // persistent dominance kernels, 4 waves per workgroup; at least 16 workgroups
    // so that every ticket class has a wave
    const int n_wg = std::max(ctx->n_cu * tp.wgcu, 64);

    // ---------------------------------------------------------------- output destination
    // ids go straight to host memory: into out_ids when it is pinned (device
    // accessible), else into the context's pinned buffer and then copied
    int64_t *dst = nullptr;
    uint32_t dcap = n;
    {
        hipPointerAttribute_t pa;
        if (out_cap > 0 && hipPointerGetAttributes(&pa, out_ids) == hipSuccess && pa.type == hipMemoryTypeHost &&
            pa.devicePointer) {
            dst = (int64_t *)pa.devicePointer;
            dcap = (uint32_t)(out_cap < (int64_t)n ? out_cap : (int64_t)n);
        } else {
            (void)hipGetLastError();   // an unregistered pointer is not an error here
        }
    }
    const bool direct = dst != nullptr;
    if (!direct) {
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, ctx->ids_h, 0) != hipSuccess || !dp)
            return set_err(ctx, SKY_ERR_HIP, "pinned output buffer is not device accessible");
        dst = (int64_t *)dp;
    }
    const bool phases = (o.flags & SKY_FLAG_PHASE_TIMES) != 0;
    // Calls without stats, phase times or work counts replay a captured graph of
    // the whole launch sequence (a learned model is part of the key: its serial
    // is never reused, so a graph never outlives the buffers it bakes in). The
    // graph assumes that no run of equal x_s straddles a slice boundary (no wait
    // for the tie check); when the check fires after all, the call runs again
    // without the graph.
    const bool graph_ok = !stats && !phases && !count_work && !(o.flags & SKY_FLAG_NO_GRAPH);
    int kreps = 0;
    uint32_t *pool_ids = P<uint32_t>(ctx->cover);
    const bool sliced = kind == SKY_PART_SLICED && np > 1;
    const bool sel_sliced = sliced && np <= SKY_QSEL_MAX_P;
    const bool rnd = kind == SKY_PART_RANDOM && np > 1;
    // the launch sequence on stream s; graph: being captured
    auto enqueue = [&](hipStream_t s, bool graph) -> int {
#define PHASE(i) do { if (phases) HIP_OK(hipEventRecord(ctx->evp[i], s)); } while (0)
        kreps = 0;   // set by the representative step of this sequence
        if (!graph) HIP_OK(hipEventRecord(ctx->ev0, s));
        PHASE(0);
        // ---------------------------------------------------------------- resets
        {   // every reset of the call in one launch (dead flags of the local and merge kernels included)
            FillSet fs{};
            fs.add(ctrl, 0, C_NUM);
            fs.add(P<uint32_t>(ctx->tick), 0, (size_t)3 * SKY_TICK_SET);
            if (count_work) fs.add(P<uint32_t>(ctx->wcnt), 0, (size_t)2 * SKY_TICK_C * 8 * 2);
            fs.add(sb.ticket, 0, 1);
            fs.add(P<uint32_t>(ctx->skybits), 0, (size_t)n / 32 + 1);
            fs.add(P<uint32_t>(ctx->part_hist), 0, (size_t)np + 1);
            if (gf) fs.add(P<uint32_t>(ctx->occ), 0, SKY_MAX_GRID_CELLS / 32);
            if (o.reps != SKY_REPS_NONE) fs.add(P<uint32_t>(ctx->selhist), 0, SKY_HCOPY * 512);   // the first histogram
            fs.add(P<uint32_t>(ctx->in_u), 0, ((size_t)n + 512) / 4);
            fs.add(P<uint32_t>(ctx->udead), 0, ((size_t)n + 512) / 4);
            if (sel_sliced) fs.add(P<uint32_t>(ctx->qsel) + SKY_QSEL_ZERO, 0, sky_qsel_zero_words(np));
            HIP_OK(launch_fill_multi(fs, s));
        }

        // With representatives, the Sliced selection's passes run inside their
        // select launches (the two sweep the points in the same grid); without,
        // it has launches of its own.
        const bool rep_topk = ((o.reps == SKY_REPS_SORTED || own_scores) && o.n_reps > 0) || o.reps == SKY_REPS_LEARNED;
        const bool qsel_fused = sel_sliced && rep_topk;
        // the side stream takes work that reads only the points: the scorer's
        // scores (joined before the representatives) and a Sliced selection of
        // its own (joined before the filter). It forks after the resets, but its
        // launches are issued after the ingest's, which therefore starts first.
        const bool fork = ((sel_sliced && !qsel_fused) || learned) && !graph;
        hipStream_t s2 = fork ? ctx->side : s;
        if (fork) HIP_OK(hipEventRecord(ctx->ev_fork, s));

        // ---------------------------------------------------------------- ingest, scores
        float *score = P<float>(ctx->score);
        const bool zorder = o.presort == SKY_PRESORT_ZORDER || o.presort == SKY_PRESORT_ZORDER_SUM;
        float *zq = P<float>(ctx->zq);   // [0, 32): per-dimension lower bound and scale; then per-workgroup bounds
        HIP_OK(launch_ingest(pts, n, d, need_range ? 1 : 0, score, gf ? 1 : 0, gg, P<uint32_t>(ctx->occ), ctrl,
                             zorder ? zq + 64 : nullptr, s));

        // ---------------------------------------------------------------- side stream; Sliced boundaries (first part)
        // Up to SKY_QSEL_MAX_P slices: the first key of every slice by a radix
        // selection, and the filter assigns the slices. More slices: a rank sort on
        // x_s (id order among equal values). Either way the check whether equal
        // values straddle a slice boundary reaches the host while the GPU goes on
        // with the representatives and the filters.
        uint32_t *sbnd = P<uint32_t>(ctx->qsel) + SKY_QSEL_WORDS;
        if (fork) HIP_OK(hipStreamWaitEvent(s2, ctx->ev_fork, 0));
        if (learned) {
            rc = sky_mlp_score_internal(o.model, pts, n, d, P<float>(ctx->score2), s2);
            if (rc != SKY_OK) return set_err(ctx, rc, "MLP scoring failed");
            if (fork) HIP_OK(hipEventRecord(ctx->ev_mlp, s2));
        }
        const QselJob qjob{pts + (size_t)o.slice_dim * n, np, P<uint32_t>(ctx->qsel), sbnd, ctrl};
        if (sel_sliced) {
            if (!qsel_fused) {   // else it runs inside the representatives' select launches
                HIP_OK(launch_sliced_select(pts + (size_t)o.slice_dim * n, n, np, P<uint32_t>(ctx->qsel), sbnd, ctrl,
                                            s2));
                if (!graph) {
                    HIP_OK(hipMemcpyAsync(ctx->ctrl_h, ctrl, C_NUM * 4, hipMemcpyDeviceToHost, s2));   // only C_TIE
                    HIP_OK(hipEventRecord(ctx->ev_tie, s2));
                }
                if (fork) HIP_OK(hipEventRecord(ctx->ev_join, s2));
            }
        } else if (rnd) {
            // Random partitioning: ranks of the points' draws (assigned after the filter)
            HIP_OK(launch_random_init(n, o.seed, sb.kA, sb.vA, s));
            HIP_OK(launch_radix_sort(sb, nullptr, n, 0, 32, s));
        } else if (sliced) {
            HIP_OK(launch_sliced_init(pts, n, o.slice_dim, sb.kA, sb.vA, s));
            HIP_OK(launch_radix_sort(sb, nullptr, n, 0, 32, s));
            HIP_OK(launch_sliced_check(sb.kA, n, np, ctrl, s));
            if (!graph) {
                HIP_OK(hipMemcpyAsync(ctx->ctrl_h, ctrl, C_NUM * 4, hipMemcpyDeviceToHost, s));
                HIP_OK(hipEventRecord(ctx->ev_tie, s));
            }
        }

        if (learned && fork) HIP_OK(hipStreamWaitEvent(s, ctx->ev_mlp, 0));
        if (own_scores) HIP_OK(launch_rep_scores(pts, n, d, o.reps, o.seed, P<float>(ctx->score2), s));
        const float *rep_score = o.reps == SKY_REPS_LEARNED || own_scores ? P<float>(ctx->score2) : score;
        const float *sort_score = o.presort == SKY_PRESORT_LEARNED ? P<float>(ctx->score2) : score;
        if (gf) HIP_OK(launch_grid_dom(P<uint32_t>(ctx->occ), P<uint32_t>(ctx->gdom), gg, s));

        // ---------------------------------------------------------------- representatives
        PHASE(1);
        if (o.reps == SKY_REPS_SORTED || own_scores) {
            // Sorted: the n_reps smallest by (sum, id); Region and random: by their scores
            kreps = o.n_reps < (int)n ? o.n_reps : (int)n;
            HIP_OK(launch_topk(rep_score, nullptr, n, kreps, 0, ctrl, P<uint32_t>(ctx->selhist), P<uint64_t>(ctx->cand),
                               s, qsel_fused ? &qjob : nullptr));
            HIP_OK(launch_reps_finalize(pts, n, d, P<uint64_t>(ctx->cand), C_NCAND, ctrl, P<uint32_t>(ctx->rep_ids),
                                        P<uint8_t>(ctx->rep_keep), P<uint32_t>(ctx->krec), s));
        } else if (o.reps == SKY_REPS_LEARNED) {
            // Learned: a pool of the smallest by sum and by learned score, then
            // the mix of the two that covers the most of a stride sample is used
            kreps = o.n_reps < (int)n ? o.n_reps : (int)n;
            const int kp = SKY_POOL_HALF < (int)n ? SKY_POOL_HALF : (int)n;
            uint64_t *cand = P<uint64_t>(ctx->cand);
            HIP_OK(launch_topk(score, rep_score, n, kp, kp, ctrl, P<uint32_t>(ctx->selhist), cand, s,
                               qsel_fused ? &qjob : nullptr));
            HIP_OK(launch_pool_mix(pts, n, d, cand, ctrl, pool_ids, kreps, cand + 2 * SKY_MAXREPS, s));
            HIP_OK(launch_reps_finalize(pts, n, d, cand + 2 * SKY_MAXREPS, C_NPICK, ctrl, P<uint32_t>(ctx->rep_ids),
                                        P<uint8_t>(ctx->rep_keep), P<uint32_t>(ctx->krec), s));
        }

        if (qsel_fused && !graph) {   // the Sliced tie flag for the host (only C_TIE is read)
            HIP_OK(hipMemcpyAsync(ctx->ctrl_h, ctrl, C_NUM * 4, hipMemcpyDeviceToHost, s));
            HIP_OK(hipEventRecord(ctx->ev_tie, s));
        }

        // ---------------------------------------------------------------- filters + Grid/Angular ids
        PHASE(2);
        if (sel_sliced && !qsel_fused && fork) HIP_OK(hipStreamWaitEvent(s, ctx->ev_join, 0));
        HIP_OK(launch_filter(pts, n, d, gf ? 1 : 0, gg, P<uint32_t>(ctx->gdom), kreps > 0 ? 1 : 0,
                             P<uint32_t>(ctx->krec), kind, pg, ag, sel_sliced ? sbnd : nullptr, o.slice_dim,
                             P<uint32_t>(ctx->part), P<uint32_t>(ctx->part_hist), np, P<uint8_t>(ctx->alive), ctrl,
                             P<uint32_t>(ctx->wgcnt) + 8192, s));
        if (stats) HIP_OK(launch_sum_grid(P<uint32_t>(ctx->wgcnt) + 8192, n, ctrl, s));
        uint32_t *part = P<uint32_t>(ctx->part);

        // ---------------------------------------------------------------- Sliced ids
        if (sliced && graph) {
            if (!sel_sliced) HIP_OK(launch_sliced_assign(sb.vA, n, np, part, s));   // (no tie assumed)
        } else if (sliced) {
            HIP_OK(hipEventSynchronize(ctx->ev_tie));
            const bool tie = ctx->ctrl_h[C_TIE] != 0;
            const uint32_t *order = sb.vA;
            if (tie) {
                // lexicographic order (x_s, x_0, .., x_{d-1} without s, id), but only for the
                // runs of equal x_s that straddle a slice boundary; the selection gave no
                // order, so it first needs the stable sort by x_s
                if (sel_sliced) {
                    HIP_OK(launch_sliced_init(pts, n, o.slice_dim, sb.kA, sb.vA, s));
                    HIP_OK(launch_radix_sort(sb, nullptr, n, 0, 32, s));
                }
                uint32_t *goff = P<uint32_t>(ctx->poff2);   // one instance: [0, n)
                HIP_OK(launch_fill_u32(goff, 0, 1, s));
                HIP_OK(launch_fill_u32(goff + 1, n, 1, s));
                uint32_t *ord = P<uint32_t>(ctx->wpos);
                HIP_OK(launch_tie_refine(sb, pts, n, d, o.slice_dim, nullptr, goff, 1, np, 32, P<uint8_t>(ctx->udead),
                                         P<uint32_t>(ctx->in_u), P<uint32_t>(ctx->sid), ord, ctrl, s));
                // flags and counts were kept in the dead-flag arrays: clear them again
                HIP_OK(launch_fill_u32(P<uint32_t>(ctx->udead), 0, ((size_t)n + 512) / 4, s));
                HIP_OK(launch_fill_u32(P<uint32_t>(ctx->in_u), 0, ((size_t)n + 512) / 4, s));
                order = ord;
            }
            if (tie || !sel_sliced) HIP_OK(launch_sliced_assign(order, n, np, part, s));   // else the filter assigned
        } else if (rnd) {
            HIP_OK(launch_sliced_assign(sb.vA, n, np, part, s));   // rank r -> floor(r p / n)
        } else if (kind == SKY_PART_NONE || ((kind == SKY_PART_SLICED || kind == SKY_PART_RANDOM) && np == 1)) {
            HIP_OK(launch_fill_u32(part, 0, n, s));
        }

        // ---------------------------------------------------------------- representatives per partition
        // They need every point's partition, so they come after the ids; the
        // filter then runs again with them (same ids, same Grid Filtering).
        if (o.reps == SKY_REPS_SORTED_PART) {
            kreps = kp_part * np;
            HIP_OK(launch_part_reps(score, part, n, kp_part, np > 1 ? bits_for((uint32_t)np) : 0, sb, ctrl,
                                    P<uint64_t>(ctx->cand), s));
            HIP_OK(launch_reps_finalize(pts, n, d, P<uint64_t>(ctx->cand), C_NCAND, ctrl, P<uint32_t>(ctx->rep_ids),
                                        P<uint8_t>(ctx->rep_keep), P<uint32_t>(ctx->krec), s));
            if (kind == SKY_PART_GRID || kind == SKY_PART_ANGULAR)
                HIP_OK(launch_fill_u32(P<uint32_t>(ctx->part_hist), 0, (size_t)np, s));
            // (no slice boundaries: the slices are final, tie refinement included)
            HIP_OK(launch_filter(pts, n, d, gf ? 1 : 0, gg, P<uint32_t>(ctx->gdom), 1, P<uint32_t>(ctx->krec), kind, pg,
                                 ag, nullptr, o.slice_dim, part, P<uint32_t>(ctx->part_hist), np,
                                 P<uint8_t>(ctx->alive), ctrl, P<uint32_t>(ctx->wgcnt) + 8192, s));
        }

        // ---------------------------------------------------------------- presort within partitions
        PHASE(3);
        const int pbits = np > 1 ? bits_for((uint32_t)np) : 0;
        const int kbits = presort_wide(o.presort, d) ? 64 : presort_kbits(pbits);
        const bool tie = presort_tie(o.presort);
        const int kbits_all = kbits + (tie ? 32 : 0);   // width of the sorted key
        if (zorder) HIP_OK(launch_zorder_scale(zq + 64, n, d, kbits - pbits, zq, s));
        const int k32 = kbits_all <= 32 ? 1 : 0;   // keys of at most 32 bits travel as 32-bit words
        HIP_OK(launch_emit_keys(sort_score, zorder ? zq : nullptr, pts, n, d, P<uint8_t>(ctx->alive), part, pbits,
                                P<uint32_t>(ctx->wgcnt), sb.kA, sb.vA, ctrl, s,
                                P<uint32_t>(ctx->urec), P<uint32_t>(ctx->uid), kbits, tie ? 1 : 0, k32));
        if (k32)
            HIP_OK(launch_radix_sort32(sb, ctrl + C_NSURV, n, 0, kbits_all, s));
        else
            HIP_OK(launch_radix_sort(sb, ctrl + C_NSURV, n, 0, kbits_all, s));
        HIP_OK(launch_gather(pts, n, d, sb.kA, sb.vA, ctrl + C_NSURV, n, pbits, np, P<uint32_t>(ctx->rec),
                             P<uint32_t>(ctx->sid), P<uint64_t>(ctx->skey), P<uint32_t>(ctx->poff), s,
                             P<uint32_t>(ctx->urec), P<uint32_t>(ctx->uid), kbits_all, k32));
        HIP_OK(launch_block_min(d, P<uint32_t>(ctx->rec), P<uint64_t>(ctx->skey), ctrl + C_NSURV, n,
                                P<uint32_t>(ctx->bmin), s));

        // ---------------------------------------------------------------- local skylines
        uint8_t *dead = P<uint8_t>(ctx->in_u);
        uint32_t *gpart = P<uint32_t>(ctx->scratch);
        uint32_t *xlist = np <= SKY_XCD_MAX_NP ? gpart + max_chunks : nullptr;   // local work routed by XCD
        HIP_OK(launch_chunk_table(P<uint32_t>(ctx->poff), np, B, P<uint32_t>(ctx->nch), P<uint32_t>(ctx->st_off), gpart,
                                  ctrl, C_NCHUNK, max_chunks, s, xlist));
        PHASE(4);
        HIP_OK(launch_local_sky(d, tp.lppl, tp.lseg, P<uint32_t>(ctx->rec), P<uint64_t>(ctx->skey),
                                P<uint32_t>(ctx->poff), P<uint32_t>(ctx->bmin), P<uint32_t>(ctx->st_off), gpart, xlist, ctrl,
                                P<uint32_t>(ctx->tick), dead, wcnt_l, n_wg, n, s));
        PHASE(5);

        // ---------------------------------------------------------------- merge
        uint32_t *skybits = P<uint32_t>(ctx->skybits);
        if (np == 1) {
            PHASE(6);
            PHASE(7);
            HIP_OK(launch_mark_alive(dead, P<uint32_t>(ctx->sid), ctrl + C_NSURV, n, skybits, s));
        } else {
            // NoSeq with a small chunk table: the union's offsets come from the table's launch
            const bool u_in_table = o.merge == SKY_MERGE_NOSEQ && chunk_table_fuses(np, max_chunks);
            HIP_OK(launch_union(d, dead, ctrl + C_NSURV, n, P<uint32_t>(ctx->rec), P<uint32_t>(ctx->sid),
                                P<uint64_t>(ctx->skey), P<uint32_t>(ctx->poff), np, P<uint32_t>(ctx->wgcnt),
                                P<uint32_t>(ctx->wpos), P<uint32_t>(ctx->urec), P<uint32_t>(ctx->uid),
                                P<uint64_t>(ctx->ukey), P<uint32_t>(ctx->upoff), ctrl, P<int64_t>(ctx->lsizes), s,
                                !u_in_table));
            if (o.merge == SKY_MERGE_NOSEQ) {
                if (u_in_table) {
                    const UnionOffsets uo{P<uint32_t>(ctx->wpos), ctrl + C_NSURV, P<uint32_t>(ctx->upoff),
                                          P<int64_t>(ctx->lsizes)};
                    HIP_OK(launch_chunk_table(P<uint32_t>(ctx->poff), np, 64 * tp.mppl, P<uint32_t>(ctx->nch),
                                              P<uint32_t>(ctx->st_off), gpart, ctrl, C_NCHUNK2, max_chunks, s,
                                              nullptr, &uo));
                } else {
                    HIP_OK(launch_chunk_table(P<uint32_t>(ctx->upoff), np, 64 * tp.mppl, P<uint32_t>(ctx->nch),
                                              P<uint32_t>(ctx->st_off), gpart, ctrl, C_NCHUNK2, max_chunks, s));
                }
                HIP_OK(launch_block_min(d, P<uint32_t>(ctx->urec), P<uint64_t>(ctx->ukey), ctrl + C_NU, n,
                                        P<uint32_t>(ctx->ubmin), s));
                PHASE(6);
                HIP_OK(launch_merge_noseq(d, tp.mppl, tp.mseg, P<uint32_t>(ctx->urec), P<uint32_t>(ctx->ubmin),
                                          P<uint64_t>(ctx->ukey), P<uint32_t>(ctx->uid), P<uint32_t>(ctx->upoff),
                                          P<uint32_t>(ctx->st_off), gpart, np, np, kind, pg, ctrl, P<uint32_t>(ctx->tick) + SKY_TICK_SET,
                                          P<uint8_t>(ctx->udead), wcnt_m, skybits, n, n_wg, s));
                PHASE(7);
                HIP_OK(launch_mark_alive(P<uint8_t>(ctx->udead), P<uint32_t>(ctx->uid), ctrl + C_NU, n, skybits, s));
            } else {
                // final round Sky(u): u sorted by its presort key is one partition for the local-skyline kernel
                HIP_OK(launch_u_sort_prep(P<uint64_t>(ctx->ukey), ctrl + C_NU, n, sb.kA, sb.vA, s));
                HIP_OK(launch_radix_sort(sb, ctrl + C_NU, n, 0, kbits_all, s));
                HIP_OK(launch_u_regather(d, P<uint32_t>(ctx->urec), P<uint32_t>(ctx->uid), sb.vA, ctrl + C_NU, n,
                                         P<uint32_t>(ctx->rec), P<uint32_t>(ctx->sid), P<uint32_t>(ctx->poff2), s));
                HIP_OK(launch_chunk_table(P<uint32_t>(ctx->poff2), 1, B, P<uint32_t>(ctx->nch), P<uint32_t>(ctx->st_off),
                                          gpart, ctrl, C_NCHUNK, max_chunks, s));
                HIP_OK(launch_fill_u32(P<uint32_t>(ctx->in_u), 0, ((size_t)n + 512) / 4, s));
                HIP_OK(launch_block_min(d, P<uint32_t>(ctx->rec), sb.kA, ctrl + C_NU, n, P<uint32_t>(ctx->bmin), s));
                PHASE(6);
                HIP_OK(launch_local_sky(d, tp.lppl, tp.lseg, P<uint32_t>(ctx->rec), sb.kA, P<uint32_t>(ctx->poff2),
                                        P<uint32_t>(ctx->bmin), P<uint32_t>(ctx->st_off), gpart, nullptr, ctrl,
                                        P<uint32_t>(ctx->tick) + 2 * SKY_TICK_SET, dead, wcnt_m, n_wg, n, s));
                PHASE(7);
                HIP_OK(launch_mark_alive(dead, P<uint32_t>(ctx->sid), ctrl + C_NU, n, skybits, s));
            }
        }

        // ---------------------------------------------------------------- output (phase 7 began at the marking)
        HIP_OK(launch_output(skybits, n, P<uint32_t>(ctx->wgcnt), dst, dcap, ctrl, s));
        if (!graph) HIP_OK(hipEventRecord(ctx->ev1, s));
        HIP_OK(hipMemcpyAsync(ctx->ctrl_h, ctrl, C_NUM * 4, hipMemcpyDeviceToHost, s));
        if (stats) {
            HIP_OK(hipMemcpyAsync(ctx->lsizes_h, ctx->lsizes.p, (size_t)np * 8, hipMemcpyDeviceToHost, s));
            HIP_OK(hipMemcpyAsync(ctx->poff_h, ctx->poff.p, (size_t)(np + 1) * 4, hipMemcpyDeviceToHost, s));
            HIP_OK(hipMemcpyAsync(ctx->phist_h, ctx->part_hist.p, (size_t)np * 4, hipMemcpyDeviceToHost, s));
            if (kreps) {
                HIP_OK(hipMemcpyAsync(ctx->repids_h, ctx->rep_ids.p, SKY_MAXREPS * 4, hipMemcpyDeviceToHost, s));
                if (o.reps == SKY_REPS_LEARNED)
                    HIP_OK(hipMemcpyAsync(ctx->repids_h + SKY_MAXREPS, pool_ids, 2 * SKY_POOL_HALF * 4,
                                          hipMemcpyDeviceToHost, s));
                HIP_OK(hipMemcpyAsync(ctx->repkeep_h, ctx->rep_keep.p, SKY_MAXREPS, hipMemcpyDeviceToHost, s));
            }
        }
        if (stats && count_work)
            HIP_OK(hipMemcpyAsync(ctx->wcnt_h, ctx->wcnt.p, (size_t)2 * SKY_TICK_C * 8 * 8, hipMemcpyDeviceToHost, s));
        return SKY_OK;
#undef PHASE
    };

    bool done = false;
    if (graph_ok) {
        GraphKey key{};
        key.pts = pts;
        key.n = n;
        key.d = d;
        key.kind = kind;
        key.p = np;
        key.slice_dim = o.slice_dim;
        key.reps = o.reps;
        key.n_reps = o.n_reps;
        key.gf = gf ? 1 : 0;
        key.gf_m = o.grid_filter_m;
        key.merge = o.merge;
        key.presort = o.presort;
        key.seed = o.seed;
        key.model = learned ? sky_mlp_serial(o.model) : 0;
        for (int k = 0; k < SKY_MAXD; ++k) key.m[k] = o.m_per_dim[k];
        key.dst = dst;
        key.dcap = dcap;
        key.gen = ctx->gen;
        key.tp = tp;
        hipGraphExec_t ex = nullptr;
        for (auto &g : ctx->graphs)
            if (g.first == key) ex = g.second;
        if (!ex) {
            // capture on the context's own stream (the caller's may be the null stream)
            hipGraph_t gph = nullptr;
            int rcg = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed) == hipSuccess ? SKY_OK : SKY_ERR_HIP;
            if (rcg == SKY_OK) {
                rcg = enqueue(ctx->cap, true);
                if (hipStreamEndCapture(ctx->cap, &gph) != hipSuccess || !gph) rcg = SKY_ERR_HIP;
            }
            if (rcg == SKY_OK && hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0) != hipSuccess) {
                ex = nullptr;
                rcg = SKY_ERR_HIP;
            }
            if (gph) hipGraphDestroy(gph);
            (void)hipGetLastError();
            ctx->err.clear();   // a failed capture falls back to the launches below
            if (ex) {
                if (ctx->graphs.size() >= SKY_MAX_GRAPHS) {
                    hipGraphExecDestroy(ctx->graphs.front().second);
                    ctx->graphs.erase(ctx->graphs.begin());
                }
                ctx->graphs.emplace_back(key, ex);
            }
        }
        if (ex) {
            HIP_OK(hipGraphLaunch(ex, s));
            HIP_OK(hipStreamSynchronize(s));
            done = !(sliced && ctx->ctrl_h[C_TIE]);   // a tie: the assumption failed, run again
        }
    }
    if (!done) {
        if ((rc = enqueue(s, false)) != SKY_OK) return rc;
        HIP_OK(hipStreamSynchronize(s));
    }
    const uint32_t err = ctx->ctrl_h[C_ERR];
    if (err & 1u) return set_err(ctx, SKY_ERR_NONFINITE, "input holds a NaN or infinite coordinate");
    if (err & 2u) return set_err(ctx, SKY_ERR_RANGE, "a coordinate lies outside [0,1], which this option needs");
    const uint32_t nsky = ctx->ctrl_h[C_NSKY];
    *out_n = nsky;
    if ((int64_t)nsky > out_cap)
        return set_err(ctx, SKY_ERR_CAPACITY, "output capacity %lld < skyline size %u", (long long)out_cap, nsky);
    if (!direct && nsky) memcpy(out_ids, ctx->ids_h, (size_t)nsky * 8);

    if (stats) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        stats->ms_total = ms;
        if (phases) {
            HIP_OK(hipEventRecord(ctx->evp[8], s));
            HIP_OK(hipEventSynchronize(ctx->evp[8]));
            for (int i = 0; i < 8; ++i) {
                float t = 0.f;
                hipEventElapsedTime(&t, ctx->evp[i], ctx->evp[i + 1]);
                stats->ms_phase[i] = t;
            }
        }
        if (count_work)
            for (int kk = 0; kk < 2; ++kk)
                for (int c = 0; c < SKY_TICK_C; ++c) {
                    stats->work[2 * kk] += (int64_t)ctx->wcnt_h[(kk * SKY_TICK_C + c) * 8];
                    stats->work[2 * kk + 1] += (int64_t)ctx->wcnt_h[(kk * SKY_TICK_C + c) * 8 + 1];
                    stats->work[4 + kk] += (int64_t)ctx->wcnt_h[(kk * SKY_TICK_C + c) * 8 + 2];
                }
        if (count_work) stats->tests = stats->work[4] + stats->work[5];
        stats->n_after_grid = ctx->ctrl_h[C_NGRID];
        stats->n_after_reps = ctx->ctrl_h[C_NSURV];
        stats->n_reps_kept = kreps ? ctx->ctrl_h[C_NREPS_KEPT] : 0;
        stats->size_u = np == 1 ? nsky : ctx->ctrl_h[C_NU];
        stats->size_sky = nsky;
        ctx->st_part_sizes.assign(np, 0);
        ctx->st_part_kept.assign(np, 0);
        ctx->st_local.assign(np, 0);
        for (int j = 0; j < np; ++j) {
            if (kind == SKY_PART_GRID || kind == SKY_PART_ANGULAR) ctx->st_part_sizes[j] = ctx->phist_h[j];
            else if (kind == SKY_PART_SLICED || kind == SKY_PART_RANDOM) {
                const uint64_t a = ((uint64_t)j * n + np - 1) / np, b = ((uint64_t)(j + 1) * n + np - 1) / np;
                ctx->st_part_sizes[j] = (int64_t)(b - a);
            } else ctx->st_part_sizes[j] = n;
            ctx->st_part_kept[j] = (int64_t)ctx->poff_h[j + 1] - (int64_t)ctx->poff_h[j];
            ctx->st_local[j] = np == 1 ? (int64_t)nsky : ctx->lsizes_h[j];
        }
        stats->part_sizes = ctx->st_part_sizes.data();
        stats->part_kept = ctx->st_part_kept.data();
        stats->local_sizes = ctx->st_local.data();
        const int nsel = kreps ? (int)ctx->ctrl_h[C_NREPS] : 0;
        ctx->st_rep_ids.assign(nsel, -1);
        ctx->st_rep_keep.assign(nsel, 0);
        for (int r = 0; r < nsel; ++r) {
            ctx->st_rep_ids[r] = ctx->repids_h[r];
            ctx->st_rep_keep[r] = ctx->repkeep_h[r];
        }
        stats->rep_ids = ctx->st_rep_ids.data();
        stats->rep_keep = ctx->st_rep_keep.data();
        stats->n_reps = nsel;
        const int npool = o.reps == SKY_REPS_LEARNED ? 2 * SKY_POOL_HALF : 0;
        ctx->st_rep_pool.assign(npool, -1);
        for (int r = 0; r < npool; ++r) {
            const uint32_t v = ctx->repids_h[SKY_MAXREPS + r];
            ctx->st_rep_pool[r] = v == 0xFFFFFFFFu ? -1 : (int64_t)v;
        }
        stats->rep_pool = ctx->st_rep_pool.data();
        stats->n_pool = npool;
    }
    return SKY_OK;
}

// ------------------------------------------------------------------ batched skylines
// Many independent instances through one launch sequence per record width
// (instances as an outer partition level: see sky_batch.hip). Options: Sliced
// (or none), Sorted representatives (or none), NoSeq merge; Z-order or sum
// presort.
extern "C" int sky_skyline_batch(sky_ctx *ctx, const float *pts, const int64_t *ns, const int32_t *ds,
                                 int32_t n_inst, const sky_opts *opts, int64_t *out_ids, int64_t out_cap,
                                 int64_t *out_offs, sky_batch_stats *bstats, void *stream)
{
    if (!ctx) return SKY_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!opts || !out_offs || n_inst < 0 || (n_inst > 0 && (!ns || !ds)))
        return set_err(ctx, SKY_ERR_INVALID_ARG, "opts, out_offs, ns and ds are required");
    if (bstats) memset(bstats, 0, sizeof(*bstats));
    const sky_opts &o = *opts;
    if (o.partitioning != SKY_PART_SLICED && o.partitioning != SKY_PART_NONE)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "batched skylines support Sliced partitioning (or none)");
    const int p = o.partitioning == SKY_PART_NONE ? 1 : o.p;
    if (p < 1 || p > 4096) return set_err(ctx, SKY_ERR_INVALID_ARG, "batched skylines need p in [1, 4096]");
    if (o.slice_dim != 0) return set_err(ctx, SKY_ERR_INVALID_ARG, "batched Sliced partitioning slices dimension 0");
    if (o.reps != SKY_REPS_NONE && o.reps != SKY_REPS_SORTED)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "batched skylines support Sorted representatives (or none)");
    if (o.reps == SKY_REPS_SORTED && (o.n_reps < 1 || o.n_reps > SKY_MAXREPS))
        return set_err(ctx, SKY_ERR_INVALID_ARG, "n_reps must be in [1, 256]");
    if (o.merge != SKY_MERGE_NOSEQ) return set_err(ctx, SKY_ERR_INVALID_ARG, "batched skylines use the NoSeq merge");
    if (o.presort != SKY_PRESORT_ZORDER && o.presort != SKY_PRESORT_SUM)
        return set_err(ctx, SKY_ERR_INVALID_ARG, "batched skylines use the Z-order or sum presort");
    if (o.grid_filter) return set_err(ctx, SKY_ERR_INVALID_ARG, "batched skylines do not take Grid Filtering");
    if ((int64_t)n_inst * p > (1 << 24))
        return set_err(ctx, SKY_ERR_INVALID_ARG, "instances x slices must be at most 2^24");
    int64_t total = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (ds[i] < 1 || ds[i] > SKY_MAXD) return set_err(ctx, SKY_ERR_INVALID_ARG, "instance %d: d=%d", i, ds[i]);
        if (ns[i] < 0) return set_err(ctx, SKY_ERR_INVALID_ARG, "instance %d: negative size", i);
        total += ns[i];
    }
    if (total > 0 && !pts) return set_err(ctx, SKY_ERR_INVALID_ARG, "pts is NULL");
    if (out_cap > 0 && !out_ids) return set_err(ctx, SKY_ERR_INVALID_ARG, "out_ids is NULL");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, SKY_ERR_HIP, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;

    // float offsets of the instances in the packed input; groups by record width
    std::vector<int64_t> foff_all(n_inst + 1, 0);
    for (int i = 0; i < n_inst; ++i) foff_all[i + 1] = foff_all[i] + (int64_t)ds[i] * ns[i];
    std::vector<std::vector<int>> groups;
    std::vector<int> gdp;
    for (int i = 0; i < n_inst; ++i) {
        if (ns[i] == 0) continue;
        const int dp = sky_dp(ds[i]);
        size_t g = 0;
        while (g < gdp.size() && gdp[g] != dp) ++g;
        if (g == gdp.size()) { gdp.push_back(dp); groups.emplace_back(); }
        groups[g].push_back(i);
    }
    for (auto &g : groups) {
        int64_t t = 0;
        for (int i : g) t += ns[i];
        if (t >= (1ll << 31)) return set_err(ctx, SKY_ERR_INVALID_ARG, "a batch group holds 2^31 points or more");
    }
    // every group's skyline lands in the pinned buffer at the group's base:
    // instance i's group indices at istart[i], its own ids after subtracting ibase[i]
    std::vector<uint32_t> cnt_all(n_inst, 0);
    std::vector<int64_t> istart(n_inst, 0), ibase(n_inst, 0);
    {
        int rc0 = grow_pinned(ctx, 0, (size_t)total);
        if (rc0 != SKY_OK) return rc0;
    }
    size_t gbase = 0;
    float ms_total = 0.f;

    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const std::vector<int> &g = groups[gi];
        const int ng = (int)g.size();
        int dg = 0;
        uint32_t NT = 0;
        for (int i : g) { dg = ds[i] > dg ? ds[i] : dg; NT += (uint32_t)ns[i]; }
        const int np = ng * p;
        const int DP = sky_dp(dg);
        const TuneParams tp = tune_for(ctx, dg, NT);
        const int B = 64 * tp.lppl;
        const uint32_t max_chunks = NT / (uint32_t)(LS_MIN_CHUNK) + (uint32_t)np + 2;
        const int G = sort_groups(NT);
        int rc;
#define ENS(b, bytes) if ((rc = ensure(ctx, ctx->b, (bytes))) != SKY_OK) return rc
        ENS(ctrl, C_NUM * 4);
        ENS(score, (size_t)NT * 4);
        ENS(part, (size_t)NT * 4);
        ENS(alive, (size_t)NT);
        ENS(kA, (size_t)NT * 8);
        ENS(kB, (size_t)NT * 8);
        ENS(vA, (size_t)NT * 4);
        ENS(vB, (size_t)NT * 4);
        ENS(shist, ((size_t)256 * 1024 + 1024 + 64) * 4);
        ENS(wgcnt, (size_t)(NT / 4096 + 8192 + 4200) * 4);
        ENS(rec, (size_t)NT * DP * 4);
        ENS(wpos, (size_t)NT * 4);
        ENS(sid, (size_t)NT * 4);
        ENS(skey, (size_t)NT * 8);
        ENS(in_u, (size_t)NT + 512);
        ENS(poff, (size_t)(np + 2) * 4);
        ENS(nch, (size_t)(np + 1) * 4);
        ENS(st_off, (size_t)(np + 2) * 4);
        ENS(scratch, ((size_t)2 * max_chunks + np + 8) * 4);
        ENS(urec, (size_t)NT * DP * 4);
        ENS(uid, (size_t)NT * 4);
        ENS(ukey, (size_t)NT * 8);
        ENS(upoff, (size_t)(np + 2) * 4);
        ENS(lsizes, (size_t)(np + 1) * 8);
        ENS(skybits, ((size_t)NT / 32 + 1) * 4);
        ENS(udead, (size_t)NT + 512);
        ENS(bmin, sky_corner_words(NT, DP) * 4);
        ENS(ubmin, sky_corner_words(NT, DP) * 4);
        ENS(zq, (size_t)(2 * 16 * SKY_INGEST_MAX_WG + 64) * 4);
        ENS(tick, (size_t)3 * SKY_TICK_SET * 4);
        ENS(bpts, (size_t)NT * dg * 4);
        ENS(binst, (size_t)NT * 4);
        ENS(bkrec, (size_t)ng * SKY_MAXREPS * DP * 4);
        ENS(bmeta, (size_t)ng * 8 + (size_t)(ng + 1) * 4 + (size_t)ng * 4 + (size_t)ng * 4 + (size_t)ng * 4 + 64);
#undef ENS
        if ((rc = grow_pinned(ctx, (size_t)np, 0)) != SKY_OK) return rc;
        const size_t meta_bytes = (size_t)ng * 8 + (size_t)(ng + 1) * 4 + (size_t)ng * 4;
        if (ctx->bmeta_h_cap < meta_bytes + (size_t)ng * 4) {
            if (ctx->bmeta_h) hipHostFree(ctx->bmeta_h);
            ctx->bmeta_h = nullptr;
            ctx->bmeta_h_cap = 0;
            if (hipHostMalloc((void **)&ctx->bmeta_h, meta_bytes + (size_t)ng * 4 + 64, hipHostMallocDefault) !=
                hipSuccess)
                return set_err(ctx, SKY_ERR_OOM, "pinned allocation failed");
            ctx->bmeta_h_cap = meta_bytes + (size_t)ng * 4;
        }
        // per-instance metadata: foff (int64), goff (u32, ng+1), gd (i32); then counts back
        char *mh = ctx->bmeta_h;
        int64_t *foff_h = (int64_t *)mh;
        uint32_t *goff_h = (uint32_t *)(mh + (size_t)ng * 8);
        int32_t *gd_h = (int32_t *)(mh + (size_t)ng * 8 + (size_t)(ng + 1) * 4);
        uint32_t *cnt_h = (uint32_t *)(mh + meta_bytes);
        uint32_t run = 0;
        for (int k = 0; k < ng; ++k) {
            foff_h[k] = foff_all[g[k]];
            goff_h[k] = run;
            gd_h[k] = ds[g[k]];
            run += (uint32_t)ns[g[k]];
        }
        goff_h[ng] = run;
        char *md = (char *)ctx->bmeta.p;
        const int64_t *foff_d = (const int64_t *)md;
        const uint32_t *goff_d = (const uint32_t *)(md + (size_t)ng * 8);
        const int32_t *gd_d = (const int32_t *)(md + (size_t)ng * 8 + (size_t)(ng + 1) * 4);
        uint32_t *nk_d = (uint32_t *)(md + meta_bytes);
        uint32_t *cnt_d = nk_d + ng;
        uint32_t *ctrl = P<uint32_t>(ctx->ctrl);
        SortBufs sb{P<uint64_t>(ctx->kA), P<uint64_t>(ctx->kB), P<uint32_t>(ctx->vA), P<uint32_t>(ctx->vB),
                    P<uint32_t>(ctx->shist), P<uint32_t>(ctx->shist) + 256 * 1024,
                    P<uint32_t>(ctx->shist) + 256 * 1024 + 1024, G};
        const int n_wg = std::max(ctx->n_cu * tp.wgcu, 64);
        float *gpts = P<float>(ctx->bpts);
        uint32_t *inst = P<uint32_t>(ctx->binst);
        const int ib = ng > 1 ? bits_for((uint32_t)ng) : 1;
        const int ibits = ((32 + ib + 15) / 16) * 16;   // an even number of 8-bit passes

        HIP_OK(hipEventRecord(ctx->ev0, s));
        HIP_OK(hipMemcpyAsync(md, mh, meta_bytes, hipMemcpyHostToDevice, s));
        HIP_OK(launch_fill_u32(ctrl, 0, C_NUM, s));
        HIP_OK(launch_fill_u32(P<uint32_t>(ctx->tick), 0, (size_t)3 * SKY_TICK_SET, s));
        HIP_OK(launch_fill_u32(sb.ticket, 0, 1, s));   // the sorts' scan ticket (fresh memory holds anything)
        HIP_OK(launch_fill_u32(P<uint32_t>(ctx->skybits), 0, (size_t)NT / 32 + 1, s));
        HIP_OK(launch_batch_pack(pts, foff_d, goff_d, gd_d, ng, NT, dg, gpts, inst, s));
        const bool zorder = o.presort == SKY_PRESORT_ZORDER || o.presort == SKY_PRESORT_ZORDER_SUM;
        float *zq = P<float>(ctx->zq);
        float *score = P<float>(ctx->score);
        GridSpec gg{};
        gg.d = dg;
        HIP_OK(launch_ingest(gpts, NT, dg, 0, score, 0, gg, nullptr, ctrl, zorder ? zq + 64 : nullptr, s));
        // Sorted representatives of every instance: sort by (instance, sum, index)
        uint8_t *alive = P<uint8_t>(ctx->alive);
        if (o.reps == SKY_REPS_SORTED) {
            HIP_OK(launch_batch_keys(inst, score, NT, sb.kA, sb.vA, s));
            HIP_OK(launch_radix_sort(sb, nullptr, NT, 0, ibits, s));
            HIP_OK(launch_batch_reps(gpts, NT, dg, sb.vA, goff_d, ng, o.n_reps, P<uint32_t>(ctx->bkrec), nk_d, s));
            HIP_OK(launch_batch_filter(gpts, NT, dg, inst, P<uint32_t>(ctx->bkrec), nk_d, alive, s));
        } else {
            HIP_OK(launch_fill_u32((uint32_t *)alive, 0x01010101u, ((size_t)NT + 3) / 4, s));
        }
        // Sliced ranks inside every instance: sort by (instance, x_0, index)
        uint32_t *part = P<uint32_t>(ctx->part);
        if (p > 1) {
            HIP_OK(launch_batch_keys(inst, gpts, NT, sb.kA, sb.vA, s));
            HIP_OK(launch_radix_sort(sb, nullptr, NT, 0, ibits, s));
            HIP_OK(launch_batch_sliced_check(sb.kA, goff_d, ng, p, ctrl, s));
            HIP_OK(hipMemcpyAsync(ctx->ctrl_h, ctrl, C_NUM * 4, hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            const uint32_t *order = sb.vA;
            if (ctx->ctrl_h[C_TIE]) {
                // lexicographic (instance, x_0, x_1, .., x_{d-1}, index), but only for
                // the runs of equal (instance, x_0) that straddle a slice boundary
                uint32_t *ord = P<uint32_t>(ctx->wpos);
                HIP_OK(launch_fill_u32(P<uint32_t>(ctx->udead), 0, ((size_t)NT + 3) / 4, s));
                HIP_OK(launch_tie_refine(sb, gpts, NT, dg, 0, inst, goff_d, ng, p, ibits, P<uint8_t>(ctx->udead),
                                         P<uint32_t>(ctx->in_u), P<uint32_t>(ctx->sid), ord, ctrl, s));
                order = ord;
            }
            HIP_OK(launch_batch_sliced_assign(order, inst, goff_d, NT, p, part, s));
        } else {
            // one partition per instance
            HIP_OK(hipMemcpyAsync(part, inst, (size_t)NT * 4, hipMemcpyDeviceToDevice, s));
        }
        // presort, local skylines, union, NoSeq merge inside each instance
        const int pbits = np > 1 ? bits_for((uint32_t)np) : 0;
        const int kbits = presort_kbits(pbits);
        if (kbits - pbits < 1) return set_err(ctx, SKY_ERR_INVALID_ARG, "too many partitions in one batch");
        if (zorder) HIP_OK(launch_zorder_scale(zq + 64, NT, dg, kbits - pbits, zq, s));
        // (kbits <= 32: the keys travel as 32-bit words)
        HIP_OK(launch_emit_keys(score, zorder ? zq : nullptr, gpts, NT, dg, alive, part, pbits,
                                P<uint32_t>(ctx->wgcnt), sb.kA, sb.vA, ctrl, s, P<uint32_t>(ctx->urec),
                                P<uint32_t>(ctx->uid), kbits, 0, 1));
        HIP_OK(launch_radix_sort32(sb, ctrl + C_NSURV, NT, 0, kbits, s));
        HIP_OK(launch_gather(gpts, NT, dg, sb.kA, sb.vA, ctrl + C_NSURV, NT, pbits, np, P<uint32_t>(ctx->rec),
                             P<uint32_t>(ctx->sid), P<uint64_t>(ctx->skey), P<uint32_t>(ctx->poff), s,
                             P<uint32_t>(ctx->urec), P<uint32_t>(ctx->uid), kbits, 1));
        HIP_OK(launch_block_min(dg, P<uint32_t>(ctx->rec), P<uint64_t>(ctx->skey), ctrl + C_NSURV, NT,
                                P<uint32_t>(ctx->bmin), s));
        uint8_t *dead = P<uint8_t>(ctx->in_u);
        uint32_t *gpart = P<uint32_t>(ctx->scratch);
        HIP_OK(launch_chunk_table(P<uint32_t>(ctx->poff), np, B, P<uint32_t>(ctx->nch), P<uint32_t>(ctx->st_off),
                                  gpart, ctrl, C_NCHUNK, max_chunks, s));
        HIP_OK(launch_fill_u32(P<uint32_t>(ctx->in_u), 0, ((size_t)NT + 512) / 4, s));
        HIP_OK(launch_local_sky(dg, tp.lppl, tp.lseg, P<uint32_t>(ctx->rec), P<uint64_t>(ctx->skey),
                                P<uint32_t>(ctx->poff), P<uint32_t>(ctx->bmin), P<uint32_t>(ctx->st_off), gpart, nullptr, ctrl,
                                P<uint32_t>(ctx->tick), dead, nullptr, n_wg, NT, s));
        uint32_t *skybits = P<uint32_t>(ctx->skybits);
        if (p == 1) {
            HIP_OK(launch_mark_alive(dead, P<uint32_t>(ctx->sid), ctrl + C_NSURV, NT, skybits, s));
        } else {
            HIP_OK(launch_union(dg, dead, ctrl + C_NSURV, NT, P<uint32_t>(ctx->rec), P<uint32_t>(ctx->sid),
                                P<uint64_t>(ctx->skey), P<uint32_t>(ctx->poff), np, P<uint32_t>(ctx->wgcnt),
                                P<uint32_t>(ctx->wpos), P<uint32_t>(ctx->urec), P<uint32_t>(ctx->uid),
                                P<uint64_t>(ctx->ukey), P<uint32_t>(ctx->upoff), ctrl, P<int64_t>(ctx->lsizes), s));
            HIP_OK(launch_chunk_table(P<uint32_t>(ctx->upoff), np, 64 * tp.mppl, P<uint32_t>(ctx->nch),
                                      P<uint32_t>(ctx->st_off), gpart, ctrl, C_NCHUNK2, max_chunks, s));
            HIP_OK(launch_fill_u32(P<uint32_t>(ctx->udead), 0, ((size_t)NT + 512) / 4, s));
            HIP_OK(launch_block_min(dg, P<uint32_t>(ctx->urec), P<uint64_t>(ctx->ukey), ctrl + C_NU, NT,
                                    P<uint32_t>(ctx->ubmin), s));
            GridSpec pg{};
            HIP_OK(launch_merge_noseq(dg, tp.mppl, tp.mseg, P<uint32_t>(ctx->urec), P<uint32_t>(ctx->ubmin),
                                      P<uint64_t>(ctx->ukey), P<uint32_t>(ctx->uid), P<uint32_t>(ctx->upoff),
                                      P<uint32_t>(ctx->st_off), gpart, np, p, SKY_PART_SLICED, pg, ctrl, P<uint32_t>(ctx->tick) + SKY_TICK_SET,
                                      P<uint8_t>(ctx->udead), nullptr, skybits, NT, n_wg, s));
            HIP_OK(launch_mark_alive(P<uint8_t>(ctx->udead), P<uint32_t>(ctx->uid), ctrl + C_NU, NT, skybits, s));
        }
        // ascending group indices of the skyline into pinned host memory, and per-instance counts
        void *dp_ = nullptr;
        if (hipHostGetDevicePointer(&dp_, ctx->ids_h, 0) != hipSuccess || !dp_)
            return set_err(ctx, SKY_ERR_HIP, "pinned output buffer is not device accessible");
        HIP_OK(launch_output(skybits, NT, P<uint32_t>(ctx->wgcnt), (int64_t *)dp_ + gbase, NT, ctrl, s));
        HIP_OK(launch_batch_counts(skybits, goff_d, ng, cnt_d, s));
        HIP_OK(hipEventRecord(ctx->ev1, s));
        HIP_OK(hipMemcpyAsync(cnt_h, cnt_d, (size_t)ng * 4, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(ctx->ctrl_h, ctrl, C_NUM * 4, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (ctx->ctrl_h[C_ERR] & 1u) return set_err(ctx, SKY_ERR_NONFINITE, "input holds a NaN or infinite coordinate");
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        ms_total += ms;
        const uint32_t nsky = ctx->ctrl_h[C_NSKY];
        uint32_t pos = 0;
        for (int k = 0; k < ng; ++k) {
            istart[g[k]] = (int64_t)(gbase + pos);
            ibase[g[k]] = goff_h[k];
            cnt_all[g[k]] = cnt_h[k];
            pos += cnt_h[k];
        }
        if (pos != nsky) return set_err(ctx, SKY_ERR_HIP, "per-instance skyline counts do not add up");
        gbase += nsky;
    }
    // assemble in instance order
    int64_t run = 0;
    for (int i = 0; i < n_inst; ++i) { out_offs[i] = run; run += cnt_all[i]; }
    out_offs[n_inst] = run;
    if (run > out_cap) return set_err(ctx, SKY_ERR_CAPACITY, "output capacity %lld < %lld ids", (long long)out_cap,
                                      (long long)run);
    for (int i = 0; i < n_inst; ++i) {   // group index -> the instance's own index
        if (cnt_all[i] == 0) continue;
        const int64_t *src = ctx->ids_h + istart[i];
        int64_t *dst = out_ids + out_offs[i];
        const int64_t b = ibase[i];
        for (uint32_t q = 0; q < cnt_all[i]; ++q) dst[q] = src[q] - b;
    }
    if (bstats) {
        bstats->n_total = total;
        bstats->size_sky = run;
        bstats->n_groups = (int32_t)groups.size();
        bstats->ms_total = ms_total;
    }
    return SKY_OK;
}

// ------------------------------------------------------------------ tuning table and autotuner
static const char *TUNE_MAGIC = "skyline-tune";

extern "C" void sky_tune_default(int32_t d, sky_tune_params *out)
{
    if (!out) return;
    const TuneParams t = tune_builtin(d < 1 ? 1 : d);
    *out = sky_tune_params{t.lppl, t.lseg, t.mppl, t.mseg, t.wgcu};
}

static TuneParams from_pub(const sky_tune_params &p)
{
    return TuneParams{p.local_ppl, p.local_seg, p.merge_ppl, p.merge_seg, p.wg_per_cu};
}

static sky_tune_params to_pub(const TuneParams &t) { return sky_tune_params{t.lppl, t.lseg, t.mppl, t.mseg, t.wgcu}; }

extern "C" int sky_tune_set(sky_ctx *ctx, int32_t d, int64_t n, const sky_tune_params *params)
{
    if (!ctx) return SKY_ERR_INVALID_ARG;
    int r, b;
    if (!params || d < 1 || d > SKY_MAXD || n < 1 || !tune_slot(sky_dp(d), (uint64_t)n, &r, &b))
        return set_err(ctx, SKY_ERR_INVALID_ARG, "sky_tune_set: bad d or n");
    const TuneParams t = from_pub(*params);
    if (!tune_valid(t)) return set_err(ctx, SKY_ERR_INVALID_ARG, "sky_tune_set: a field is outside its range");
    ctx->tune[r][b] = t;
    ctx->tune_has[r][b] = true;
    return SKY_OK;
}

extern "C" int sky_tune_get(const sky_ctx *ctx, int32_t d, int64_t n, sky_tune_params *out)
{
    int r, b;
    if (!ctx || !out || d < 1 || d > SKY_MAXD || n < 0 || !tune_slot(sky_dp(d), (uint64_t)n, &r, &b))
        return SKY_ERR_INVALID_ARG;
    *out = to_pub(tune_for(ctx, d, (uint64_t)n));
    return ctx->tune_has[r][b] ? 1 : 0;
}

extern "C" void sky_tune_clear(sky_ctx *ctx)
{
    if (!ctx) return;
    for (auto &row : ctx->tune_has)
        for (bool &h : row) h = false;
}

extern "C" int sky_tune_save(const sky_ctx *ctx, const char *path)
{
    if (!ctx || !path) return SKY_ERR_INVALID_ARG;
    FILE *f = fopen(path, "w");
    if (!f) return SKY_ERR_IO;
    bool ok = fprintf(f, "%s 1 %s %d\n", TUNE_MAGIC, ctx->arch.empty() ? "unknown" : ctx->arch.c_str(),
                      ctx->n_cu) > 0;
    for (int r = 0; r < 5 && ok; ++r)
        for (int b = 0; b < 33 && ok; ++b)
            if (ctx->tune_has[r][b]) {
                const TuneParams &t = ctx->tune[r][b];
                ok = fprintf(f, "%d %d %d %d %d %d %d\n", 4 * (r + 1), b, t.lppl, t.lseg, t.mppl, t.mseg,
                             t.wgcu) > 0;
            }
    ok = (fclose(f) == 0) && ok;
    return ok ? SKY_OK : SKY_ERR_IO;
}

extern "C" int sky_tune_load(sky_ctx *ctx, const char *path)
{
    if (!ctx || !path) return SKY_ERR_INVALID_ARG;
    ctx->err.clear();
    FILE *f = fopen(path, "r");
    if (!f) return set_err(ctx, SKY_ERR_IO, "cannot open %s", path);
    char magic[32] = {}, arch[128] = {};
    int ver = 0, ncu = 0;
    const std::string want = ctx->arch.empty() ? "unknown" : ctx->arch;
    if (fscanf(f, "%31s %d %127s %d", magic, &ver, arch, &ncu) != 4 || strcmp(magic, TUNE_MAGIC) != 0 || ver != 1) {
        fclose(f);
        return set_err(ctx, SKY_ERR_INVALID_ARG, "%s is not a tuning table", path);
    }
    if (want != arch || ncu != ctx->n_cu) {
        fclose(f);
        return set_err(ctx, SKY_ERR_INVALID_ARG, "%s was tuned on %s with %d compute units, this device is %s with %d",
                       path, arch, ncu, want.c_str(), ctx->n_cu);
    }
    struct Ent { int r, b; TuneParams t; };
    std::vector<Ent> ents;
    int v[7];
    int got;
    while ((got = fscanf(f, "%d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6])) == 7) {
        const TuneParams t{v[2], v[3], v[4], v[5], v[6]};
        if (v[0] < 4 || v[0] > 20 || v[0] % 4 != 0 || v[1] < 0 || v[1] > 32 || !tune_valid(t)) {
            fclose(f);
            return set_err(ctx, SKY_ERR_INVALID_ARG, "%s: bad entry \"%d %d %d %d %d %d %d\"", path, v[0], v[1], v[2],
                           v[3], v[4], v[5], v[6]);
        }
        ents.push_back(Ent{v[0] / 4 - 1, v[1], t});
    }
    const bool at_end = got == EOF;
    fclose(f);
    if (!at_end) return set_err(ctx, SKY_ERR_INVALID_ARG, "%s: malformed entry", path);
    for (const Ent &e : ents) {
        ctx->tune[e.r][e.b] = e.t;
        ctx->tune_has[e.r][e.b] = true;
    }
    return SKY_OK;
}

// Coordinate descent over the five fields. run(t, &ms) makes one call under
// splits t and returns its status; same(t) says whether that call's result
// equals the first one's. A candidate is kept only when its median beats the
// best by more than 1%.
template <typename Run, typename Apply>
static int tune_search(sky_ctx *ctx, TuneParams start, int trials, Run run, Apply apply, TuneParams *best_out,
                       float *best_ms, float *base_ms)
{
    auto measure = [&](const TuneParams &t, float *med) -> int {
        apply(t);
        float ms = 0.f;
        int rc = run(&ms, false);   // untimed call
        if (rc != SKY_OK) return rc;
        std::vector<float> v;
        for (int k = 0; k < trials; ++k) {
            if ((rc = run(&ms, true)) != SKY_OK) return rc;
            v.push_back(ms);
        }
        std::sort(v.begin(), v.end());
        *med = v[v.size() / 2];
        return SKY_OK;
    };
    TuneParams best = start;
    float bms = 0.f;
    int rc = measure(best, &bms);
    if (rc != SKY_OK) return rc;
    if (base_ms) *base_ms = bms;
    static const int PPL[] = {1, 2, 4}, SEG[] = {256, 512, 1024, 2048, 4096}, WG[] = {2, 4, 8};
    for (int pass = 0; pass < 2; ++pass) {
        const TuneParams before = best;
        for (int field = 0; field < 5; ++field) {
            const int *vals = field == 0 || field == 2 ? PPL : field == 4 ? WG : SEG;
            const int nv = field == 0 || field == 2 ? 3 : field == 4 ? 3 : 5;
            for (int k = 0; k < nv; ++k) {
                TuneParams t = best;
                int *f = field == 0 ? &t.lppl : field == 1 ? &t.lseg : field == 2 ? &t.mppl : field == 3 ? &t.mseg
                                                                                                          : &t.wgcu;
                if (*f == vals[k]) continue;
                *f = vals[k];
                float ms = 0.f;
                if ((rc = measure(t, &ms)) != SKY_OK) return rc;
                if (ms < bms * 0.99f) { best = t; bms = ms; }
            }
        }
        if (memcmp(&before, &best, sizeof best) == 0) break;
    }
    apply(best);
    if (best_out) *best_out = best;
    if (best_ms) *best_ms = bms;
    (void)ctx;
    return SKY_OK;
}

extern "C" int sky_autotune(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const sky_opts *opts,
                            int32_t trials, sky_tune_params *best, float *best_ms, float *base_ms, void *stream)
{
    if (!ctx) return SKY_ERR_INVALID_ARG;
    if (trials < 1 || trials > 50) return set_err(ctx, SKY_ERR_INVALID_ARG, "trials must be in [1, 50]");
    int r, b;
    if (d < 1 || d > SKY_MAXD || n < 1 || !tune_slot(sky_dp(d), (uint64_t)n, &r, &b))
        return set_err(ctx, SKY_ERR_INVALID_ARG, "sky_autotune: bad d or n");
    const bool had = ctx->tune_has[r][b];
    const TuneParams saved = ctx->tune[r][b];
    std::vector<int64_t> ref, ids((size_t)n);
    int64_t ref_n = -1;
    auto run = [&](float *ms, bool timed) -> int {
        int64_t on = 0;
        sky_stats st;
        const int rc = sky_skyline(ctx, pts, n, d, opts, ids.data(), n, &on, &st, stream);
        if (rc != SKY_OK) return rc;
        if (ref_n < 0) {
            ref.assign(ids.begin(), ids.begin() + on);
            ref_n = on;
        } else if (on != ref_n || memcmp(ref.data(), ids.data(), (size_t)on * 8) != 0) {
            return set_err(ctx, SKY_ERR_INTERNAL, "sky_autotune: a candidate changed the skyline");
        }
        if (timed) *ms = st.ms_total;
        return SKY_OK;
    };
    auto apply = [&](const TuneParams &t) { ctx->tune[r][b] = t; ctx->tune_has[r][b] = true; };
    TuneParams got;
    const int rc = tune_search(ctx, tune_for(ctx, d, (uint64_t)n), trials, run, apply, &got, best_ms, base_ms);
    if (rc != SKY_OK) {
        ctx->tune[r][b] = saved;
        ctx->tune_has[r][b] = had;
        return rc;
    }
    if (best) *best = to_pub(got);
    return SKY_OK;
}

extern "C" int sky_autotune_batch(sky_ctx *ctx, const float *pts, const int64_t *ns, const int32_t *ds,
                                  int32_t n_inst, const sky_opts *opts, int32_t trials, sky_tune_params *best,
                                  float *best_ms, float *base_ms, void *stream)
{
    if (!ctx) return SKY_ERR_INVALID_ARG;
    if (trials < 1 || trials > 50) return set_err(ctx, SKY_ERR_INVALID_ARG, "trials must be in [1, 50]");
    if (n_inst < 1 || !ns || !ds) return set_err(ctx, SKY_ERR_INVALID_ARG, "sky_autotune_batch: no instances");
    // the table entries of the batch's launch sequences: (record width, total points)
    std::vector<int> gdp;
    std::vector<int64_t> gn;
    int64_t total = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (ds[i] < 1 || ds[i] > SKY_MAXD || ns[i] < 0)
            return set_err(ctx, SKY_ERR_INVALID_ARG, "instance %d: bad size or d", i);
        if (ns[i] == 0) continue;
        const int dp = sky_dp(ds[i]);
        size_t g = 0;
        while (g < gdp.size() && gdp[g] != dp) ++g;
        if (g == gdp.size()) { gdp.push_back(dp); gn.push_back(0); }
        gn[g] += ns[i];
        total += ns[i];
    }
    if (total == 0) return set_err(ctx, SKY_ERR_INVALID_ARG, "sky_autotune_batch: no points");
    std::vector<int> rows(gdp.size()), cols(gdp.size());
    for (size_t g = 0; g < gdp.size(); ++g)
        if (!tune_slot(gdp[g], (uint64_t)gn[g], &rows[g], &cols[g]))
            return set_err(ctx, SKY_ERR_INVALID_ARG, "sky_autotune_batch: batch group too large");
    std::vector<TuneParams> saved(gdp.size());
    std::vector<bool> had(gdp.size());
    for (size_t g = 0; g < gdp.size(); ++g) {
        saved[g] = ctx->tune[rows[g]][cols[g]];
        had[g] = ctx->tune_has[rows[g]][cols[g]];
    }
    std::vector<int64_t> ids((size_t)total), offs((size_t)n_inst + 1), ref, ref_offs;
    auto run = [&](float *ms, bool timed) -> int {
        sky_batch_stats st;
        const int rc = sky_skyline_batch(ctx, pts, ns, ds, n_inst, opts, ids.data(), total, offs.data(), &st, stream);
        if (rc != SKY_OK) return rc;
        const int64_t on = offs[n_inst];
        if (ref_offs.empty()) {
            ref.assign(ids.begin(), ids.begin() + on);
            ref_offs = offs;
        } else if (offs != ref_offs || memcmp(ref.data(), ids.data(), (size_t)on * 8) != 0) {
            return set_err(ctx, SKY_ERR_INTERNAL, "sky_autotune_batch: a candidate changed the skylines");
        }
        if (timed) *ms = st.ms_total;
        return SKY_OK;
    };
    auto apply = [&](const TuneParams &t) {
        for (size_t g = 0; g < gdp.size(); ++g) {
            ctx->tune[rows[g]][cols[g]] = t;
            ctx->tune_has[rows[g]][cols[g]] = true;
        }
    };
    // start from the entry of the largest launch sequence
    size_t gmax = 0;
    for (size_t g = 1; g < gdp.size(); ++g)
        if (gn[g] > gn[gmax]) gmax = g;
    TuneParams got;
    const int rc = tune_search(ctx, tune_for(ctx, gdp[gmax] - 2, (uint64_t)gn[gmax]), trials, run, apply, &got,
                               best_ms, base_ms);
    if (rc != SKY_OK) {
        for (size_t g = 0; g < gdp.size(); ++g) {
            ctx->tune[rows[g]][cols[g]] = saved[g];
            ctx->tune_has[rows[g]][cols[g]] = had[g];
        }
        return rc;
    }
    if (best) *best = to_pub(got);
    return SKY_OK;
}
