// Internal declarations of the HIP skyline library (gfx950). Not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/skyline.h"

#define SKY_WG 256          // threads per workgroup for most kernels (4 wave64)
#define SKY_MAXD 16
#define SKY_MAXREPS 256
// Learned representatives: a pool of SKY_POOL_HALF points by coordinate sum and
// SKY_POOL_HALF by learned score; the representatives are the mix of the two
// that covers the most of a stride sample of at most SKY_COVER_M points.
#define SKY_POOL_HALF 64
#define SKY_COVER_M 4096
// Window blocks of the dominance scans: SKY_BLK records share one lower corner.
#define SKY_BLK_SH 6
#define SKY_BLK (1u << SKY_BLK_SH)
// Each block also carries the corners of its sub-blocks of SKY_SUB records,
// stored right after the block's own corner record: SKY_CSTRIDE corner
// records (DP words each) per block.
#define SKY_SUB_SH 3
#define SKY_SUB (1u << SKY_SUB_SH)
#define SKY_NSUB (SKY_BLK >> SKY_SUB_SH)
#define SKY_CSTRIDE (1 + SKY_NSUB)
// Super-blocks of SKY_SBB blocks carry one more corner record each, stored
// after all block corners: the scans check it before the blocks' corners.
#define SKY_SBB 32
// Words of the corner buffer for n records of DP words: the block corners,
// then the super-block corners.
static inline size_t sky_block_corner_words(uint32_t n, int DP)
{
    return ((size_t)(n >> SKY_BLK_SH) + 8) * SKY_CSTRIDE * DP;
}
static inline size_t sky_corner_words(uint32_t n, int DP)
{
    return sky_block_corner_words(n, DP) + ((size_t)(n >> SKY_BLK_SH) / SKY_SBB + 2) * DP;
}
// Work tickets of the persistent dominance kernels come from SKY_TICK_C
// counters, each in its own 64-byte line (same-address atomics serialise).
#define SKY_TICK_C 64
// Accelerator dies (XCDs, each with its own L2); workgroup b runs on XCD b % 8.
#define SKY_NXCD 8
// Largest partition count for which the local-skyline work is routed by XCD.
#define SKY_XCD_MAX_NP 1024
#define SKY_TICK_SET (SKY_TICK_C * 16)
// Largest grid of the ingest kernel (its per-workgroup bounds are reduced later).
#define SKY_INGEST_MAX_WG 8192
#define SKY_MAX_GRID_CELLS 65536

// Control block: small device counters shared by the launch sequence.
enum {
    C_ERR = 0,          // bit 0: non-finite coordinate, bit 1: coordinate outside [0,1]
    C_NSURV = 1,        // points surviving grid + representative filters
    C_NGRID = 2,        // points surviving the grid filter
    C_TICKET = 3,       // work ticket of the local-skyline kernel
    C_NCHUNK = 4,       // number of chunks of the local-skyline kernel
    C_NU = 5,           // size of the union of local skylines
    C_NSKY = 6,         // skyline size
    C_TICKET2 = 7,      // work ticket of the merge kernel
    C_NREPS = 8,        // representatives selected
    C_NREPS_KEPT = 9,   // representatives kept by the self-filter
    C_SEL_K = 10,       // radix select: rank still to find (1-based)
    C_SEL_PLO = 11,     // radix select: key prefix, low word
    C_SEL_PHI = 12,     // radix select: key prefix, high word
    C_TIE = 13,         // Sliced: a run of equal slice coordinates straddles a boundary
    C_NCAND = 14,       // candidates collected by the top-k select
    C_NCHUNK2 = 15,     // number of chunks of the merge kernel
    C_MAXC = 16,        // chunk table: max chunks per partition
    C_MAXU = 17,        // largest local skyline |u_j|
    C_SEL2_K = 18,      // second radix select (learned score): rank still to find
    C_SEL2_PLO = 19,    // second radix select: key prefix, low word
    C_SEL2_PHI = 20,    // second radix select: key prefix, high word
    C_NCAND2 = 21,      // candidates collected by the second select
    C_NPICK = 22,       // representatives picked by the coverage step
    C_XG0 = 23,         // 23..30: query groups whose partition sits on XCD 0..7
    C_MIX0 = 32,        // 32..36: sample points covered by mix candidate set 0..4
    C_MIXT = 37,        // last-workgroup ticket of the mix choice
    C_NTIE = 41,        // Sliced tie refinement: points in runs that straddle a boundary
    C_NUM = 48
};

// Partition kinds, as in skyline.h.
enum { P_NONE = 0, P_GRID = 1, P_ANGULAR = 2, P_SLICED = 3, P_RANDOM = 4 };

struct GridSpec {            // a grid of cells, dimension 0 least significant
    int32_t d;
    int32_t m[SKY_MAXD];
};

#define SKY_MAX_ANG_M 16
struct AngSpec {             // Angular partitioning: thresholds T[a][k] = tan^2(k pi / (2 m_a))
    int32_t d;
    int32_t m[SKY_MAXD];
    double T[SKY_MAXD - 1][SKY_MAX_ANG_M];   // k = 1..m_a-1, m_a <= 16
};

// Order-preserving map of a float32 onto uint32 (-0 folded onto +0): for finite
// a, b: a < b  <=>  map(a) < map(b), and a == b  <=>  map(a) == map(b).
__device__ __forceinline__ uint32_t ordmap(float x)
{
    uint32_t u = __float_as_uint(x);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Last-workgroup hand-offs inside one kernel pass their data through
// device-scope atomics only: each workgroup's read-modify-write atomics return a
// value, and waiting for that value means the operation has been performed at
// the device's coherence point; the workgroup that takes the last ticket then
// reads with atomic loads. No agent-scope fence is needed, which on gfx950
// would write back the L2 in every workgroup. sky_consume(v) makes the thread
// wait for v (an empty asm statement that takes it as input).
__device__ __forceinline__ void sky_consume(uint32_t v) { asm volatile("" ::"v"(v)); }


// Record layout of a point in the AoS work buffers: DP uint32 words,
// [map(x_0) .. map(x_{d-1}), 0 ..., K_lo, K_hi], DP = roundup(d + 2, 4),
// K = sum_k map(x_k) (uint64) in the last two words. If w and t are records, w
// dominates t exactly when each of the first DP-2 words of w is <= that of t
// (padding words are 0 in both) and K(w) != K(t): with every coordinate <=,
// equal sums force equal coordinates.
static inline int sky_dp(int d) { return ((d + 2 + 3) / 4) * 4; }

// ---------------------------------------------------------------- launches
// Launch helpers return the hipError_t of their launches. Sizes passed from
// the host are upper bounds; kernels read live sizes from device counters, so
// a launch sequence never waits for the host.
#define LS_MIN_CHUNK 64        // smallest chunk of the local-skyline and merge kernels

struct SortBufs {
    uint64_t *kA, *kB;
    uint32_t *vA, *vB;
    uint32_t *hist;     // 256 * G digit counts per workgroup, scanned in place
    uint32_t *bpre;     // [1024] prefix of the scan's block totals
    uint32_t *ticket;   // [1] zero between uses
    int G;
};

// sky_prims.hip
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
struct FillSet {   // up to 12 fills of uint32 words, one launch
    uint32_t *p[12];
    uint32_t v[12];
    size_t n[12];
    int cnt;
    void add(uint32_t *ptr, uint32_t val, size_t cnt_words)
    {
        p[cnt] = ptr;
        v[cnt] = val;
        n[cnt] = cnt_words;
        ++cnt;
    }
};
hipError_t launch_fill_multi(const FillSet &f, hipStream_t s);
hipError_t launch_scan_counts(uint32_t *a, uint32_t n, uint32_t *tmp2, uint32_t *total, hipStream_t s);
int sort_groups(uint32_t n_max);
hipError_t launch_radix_sort(SortBufs &b, const uint32_t *n_dev, uint32_t n_max, int bit_lo, int bit_hi,
                             hipStream_t s);   // result in b.kA / b.vA (after an odd pass count the two
                                               // pairs of b trade places)
// The same over 32-bit keys stored in the same buffers (bit_hi <= 32).
hipError_t launch_radix_sort32(SortBufs &b, const uint32_t *n_dev, uint32_t n_max, int bit_lo, int bit_hi,
                               hipStream_t s);
void zorder_layout(int d, int zbits, int *b, int *nz);
hipError_t launch_zorder_scale(const float *bnd, uint32_t n, int d, int zbits, float *zq, hipStream_t s);
// Presort keys are kbits wide, (partition : pbits | Q : kbits - pbits): 24 bits
// (three radix passes) while Q keeps at least 16 bits, else 32 (four).
static inline int presort_kbits(int pbits) { return pbits <= 8 ? 24 : 32; }
// The Z-order presort at d >= 7 takes a 64-bit key (eight passes) instead: a
// 32-bit code leaves two or three bits per coordinate there, so record blocks
// span much of the data and the corner checks of the dominance scans, not the
// tests, dominate the local phase; 64 bits give 7 to 9 bits per coordinate.
static inline bool presort_wide(int presort, int d) { return presort == SKY_PRESORT_ZORDER && d >= 7; }
// Whether the presort key carries the tie word (the score below the Z-order
// code, 32 more key bits and radix passes), which keeps runs of equal keys short.
static inline bool presort_tie(int presort) { return presort == SKY_PRESORT_ZORDER_SUM; }
// With rec_stage / id_stage (n_max * DP and n_max words), the emission also
// writes every survivor's record and id at its compacted position and the sort
// values are those positions; the gather then reads one staged record per
// output instead of d scattered coordinates. Without, the values are input ids.
// k32: the keys are 32-bit words in the same buffer (key width <= 32), sorted by
// launch_radix_sort32 and read so by the gather.
hipError_t launch_emit_keys(const float *score, const float *zq, const float *pts, uint32_t n, int d,
                            const uint8_t *alive, const uint32_t *part, int pbits, uint32_t *wg_cnt,
                            uint64_t *keys, uint32_t *vals, uint32_t *ctrl, hipStream_t s,
                            uint32_t *rec_stage, uint32_t *id_stage, int kbits, int tie, int k32);
hipError_t launch_gather(const float *pts, uint32_t n, int d, const uint64_t *keys, const uint32_t *vals,
                         const uint32_t *n_dev, uint32_t n_max, int pbits, int np, uint32_t *rec, uint32_t *sid,
                         uint64_t *skey, uint32_t *poff, hipStream_t s, const uint32_t *rec_stage,
                         const uint32_t *id_stage, int kbits, int k32);
hipError_t launch_output(const uint32_t *skybits, uint32_t n, uint32_t *wg_cnt, int64_t *ids, uint32_t cap,
                         uint32_t *ctrl, hipStream_t s);

// sky_kernels.hip
hipError_t launch_ingest(const float *pts, uint32_t n, int d, int need_range, float *score, int gf_on,
                         const GridSpec &gg, uint32_t *occ, uint32_t *ctrl, float *bnd, hipStream_t s);
hipError_t launch_grid_dom(const uint32_t *occ, uint32_t *gdom, const GridSpec &gg, hipStream_t s);
// Pass histograms of the radix selections are kept in SKY_HCOPY copies:
// workgroup b adds into copy b % SKY_HCOPY (same-address atomics from every
// workgroup serialise), and readers sum the copies.
#define SKY_HCOPY 8
#define SKY_SEL_WORDS (3 * SKY_HCOPY * 512 + 16)   // radix-select histograms and state
struct QselJob {   // a Sliced boundary selection run inside the representatives' select passes
    const float *xs;    // x_s of the n points
    int p;              // slices, 2 .. SKY_QSEL_MAX_P
    uint32_t *qs;       // SKY_QSEL_WORDS words of state (zeroed as for launch_sliced_select)
    uint32_t *bnd;      // p - 1 boundary keys
    uint32_t *ctrl;
};
hipError_t launch_topk(const float *score, const float *score2, uint32_t n, int k, int k2, uint32_t *ctrl,
                       uint32_t *sel, uint64_t *cand, hipStream_t s, const QselJob *qj = nullptr);
hipError_t launch_pool_mix(const float *pts, uint32_t n, int d, const uint64_t *cand, uint32_t *ctrl,
                              uint32_t *pool_ids, int n_reps, uint64_t *picked, hipStream_t s);
hipError_t launch_reps_finalize(const float *pts, uint32_t n, int d, const uint64_t *cand, int count_slot,
                                uint32_t *ctrl, uint32_t *rep_ids, uint8_t *rep_keep, uint32_t *krec,
                                hipStream_t s);
hipError_t launch_filter(const float *pts, uint32_t n, int d, int gf_on, const GridSpec &gg, const uint32_t *gdom,
                         int use_reps, const uint32_t *krec, int part_kind, const GridSpec &pg, const AngSpec &ag,
                         const uint32_t *sbnd, int sdim, uint32_t *part, uint32_t *part_hist, int np,
                         uint8_t *alive, uint32_t *ctrl, uint32_t *grid_cnt, hipStream_t s);
#define SKY_QSEL_MAX_P 64                           // largest p whose slice boundaries are selected
#define SKY_QSEL_WORDS (512 + 3 * 64 * SKY_HCOPY * 256)   // selection state and three histogram buffers
// words [SKY_QSEL_ZERO, SKY_QSEL_ZERO + sky_qsel_zero_words(p)) of the state are zero when a selection starts
#define SKY_QSEL_ZERO 512
static inline size_t sky_qsel_zero_words(int p) { return (void)p, (size_t)SKY_HCOPY * 256; }
hipError_t launch_sliced_select(const float *xs, uint32_t n, int p, uint32_t *qs, uint32_t *bnd, uint32_t *ctrl,
                                hipStream_t s);
hipError_t launch_sum_grid(const uint32_t *grid_cnt, uint32_t n, uint32_t *ctrl, hipStream_t s);
// Representative scores other than the sum: kind 3 Region (-prod (1 - x_k)),
// kind 4 random (SplitMix64 draws); Random partitioning keys.
hipError_t launch_rep_scores(const float *pts, uint32_t n, int d, int kind, uint64_t seed, float *score,
                             hipStream_t s);
hipError_t launch_random_init(uint32_t n, uint64_t seed, uint64_t *keys, uint32_t *vals, hipStream_t s);
hipError_t launch_sliced_init(const float *pts, uint32_t n, int coord, uint64_t *keys, uint32_t *vals,
                              hipStream_t s);
hipError_t launch_sliced_check(const uint64_t *keys, uint32_t n, int p, uint32_t *ctrl, hipStream_t s);
hipError_t launch_sliced_assign(const uint32_t *vals, uint32_t n, int p, uint32_t *part, hipStream_t s);
// Sorted representatives per partition (reps = SKY_REPS_SORTED_PART): the kp
// smallest by (score, id) of every partition of part[0..n) into cand, count in
// ctrl[C_NCAND] (zero on entry); pbits = bits of the largest partition id.
// Uses (and sorts into) sb.
hipError_t launch_part_reps(const float *score, const uint32_t *part, uint32_t n, int kp, int pbits, SortBufs &sb,
                            uint32_t *ctrl, uint64_t *cand, hipStream_t s);

hipError_t launch_tie_refine(SortBufs &b, const float *pts, uint32_t n, int d, int sdim, const uint32_t *inst,
                             const uint32_t *goff, int ng, int p, int kbits, uint8_t *flag, uint32_t *cnt,
                             uint32_t *pos, uint32_t *order, uint32_t *ctrl, hipStream_t s);
// The chunk table and the group map run as one single-workgroup launch when
// np <= CT_FUSE_NP and g_max <= CT_FUSE_G; then the union's offsets (what
// k_union_offsets writes) can be derived in the same launch.
#define CT_FUSE_NP 1024
#define CT_FUSE_G 32768u
static inline bool chunk_table_fuses(int np, uint32_t g_max) { return np <= CT_FUSE_NP && g_max <= CT_FUSE_G; }
struct UnionOffsets {   // inputs and outputs of the union's offsets (see launch_union)
    const uint32_t *urank, *n_dev;
    uint32_t *upoff;
    int64_t *local_sizes;   // nullable
};
// With u: poff holds the partitions' offsets and the table is built over the
// union's (requires chunk_table_fuses).
hipError_t launch_chunk_table(const uint32_t *poff, int np, int B, uint32_t *nch, uint32_t *st_off, uint32_t *gpart,
                              uint32_t *ctrl, int which, uint32_t g_max, hipStream_t s, uint32_t *xlist = nullptr,
                              const UnionOffsets *u = nullptr);


// Work splits of the dominance kernels. They change the time of a call, never
// its result; the context's tuning table picks them per (record width, n).
struct TuneParams {
    int lppl;   // query points per lane, local kernel (a query group is 64 * lppl points): 1, 2 or 4
    int lseg;   // smallest window segment of a local item, records: a power of two in [256, 8192]
    int mppl;   // query points per lane, merge kernel: 1, 2 or 4
    int mseg;   // window segment of a merge item, records: a power of two in [256, 8192]
    int wgcu;   // persistent workgroups of 4 waves per compute unit: 1 .. 8
};
TuneParams tune_builtin(int d);
bool tune_valid(const TuneParams &t);

// sky_dominance.hip
hipError_t launch_local_sky(int d, int ppl, uint32_t smin, const uint32_t *raw, const uint64_t *key,
                            const uint32_t *poff,
                            const uint32_t *bmin, const uint32_t *st_off, const uint32_t *gpart,
                            const uint32_t *xlist, uint32_t *ctrl, uint32_t *tick, uint8_t *dead, uint64_t *wcnt,
                            int n_wg, uint32_t n_in, hipStream_t s);
hipError_t launch_block_min(int d, const uint32_t *rec, const uint64_t *key, const uint32_t *n_dev, uint32_t n_max,
                            uint32_t *bmin, hipStream_t s);
hipError_t launch_union(int d, const uint8_t *dead, const uint32_t *n_dev, uint32_t n_max, const uint32_t *rec,
                        const uint32_t *sid, const uint64_t *skey, const uint32_t *poff, int np, uint32_t *wg_cnt,
                        uint32_t *urank, uint32_t *urec, uint32_t *uid, uint64_t *ukey, uint32_t *upoff,
                        uint32_t *ctrl, int64_t *local_sizes, hipStream_t s, bool offsets = true);
hipError_t launch_merge_noseq(int d, int ppl, uint32_t mseg, const uint32_t *urec, const uint32_t *ubmin,
                              const uint64_t *ukey,
                              const uint32_t *uid, const uint32_t *upoff, const uint32_t *st_off,
                              const uint32_t *gpart, int np, int ppi, int part_kind, const GridSpec &pg,
                              uint32_t *ctrl,
                              uint32_t *tick, uint8_t *udead, uint64_t *wcnt, uint32_t *skybits, uint32_t n_max,
                              int n_wg, hipStream_t s);
hipError_t launch_mark_alive(const uint8_t *dead, const uint32_t *ids, const uint32_t *n_dev, uint32_t n_max,
                             uint32_t *skybits, hipStream_t s);
hipError_t launch_u_sort_prep(const uint64_t *ukey, const uint32_t *n_dev, uint32_t n_max, uint64_t *keys,
                              uint32_t *vals, hipStream_t s);
hipError_t launch_u_regather(int d, const uint32_t *urec, const uint32_t *uid, const uint32_t *vals,
                             const uint32_t *n_dev, uint32_t n_max, uint32_t *rec, uint32_t *sid, uint32_t *poff,
                             hipStream_t s);

// sky_batch.hip
hipError_t launch_batch_pack(const float *pts, const int64_t *foff, const uint32_t *goff, const int32_t *gd, int ng,
                             uint32_t NT, int dg, float *out, uint32_t *inst, hipStream_t s);
hipError_t launch_batch_keys(const uint32_t *inst, const float *v, uint32_t NT, uint64_t *keys, uint32_t *vals,
                             hipStream_t s);
hipError_t launch_batch_reps(const float *pts, uint32_t NT, int d, const uint32_t *vals, const uint32_t *goff,
                             int ng, int nreps, uint32_t *krec, uint32_t *nk, hipStream_t s);
hipError_t launch_batch_filter(const float *pts, uint32_t NT, int d, const uint32_t *inst, const uint32_t *krec,
                               const uint32_t *nk, uint8_t *alive, hipStream_t s);
hipError_t launch_batch_sliced_check(const uint64_t *keys, const uint32_t *goff, int ng, int p, uint32_t *ctrl,
                                     hipStream_t s);
hipError_t launch_batch_sliced_assign(const uint32_t *vals, const uint32_t *inst, const uint32_t *goff, uint32_t NT,
                                      int p, uint32_t *part, hipStream_t s);
hipError_t launch_batch_counts(const uint32_t *bits, const uint32_t *goff, int ng, uint32_t *cnt, hipStream_t s);
