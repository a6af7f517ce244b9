// The dominance-test kernels: local skylines with SFS semantics (Algorithm 1
// inside each partition of Algorithm 2) and the NoSeq merge (Proposition 2).
//
// Records (see sky_internal.h) hold order-preserving uint32 images of the
// coordinates plus K = their sum; w dominates t iff all coordinate words of w
// are <= those of t and K(w) != K(t). Inside a partition the points are sorted
// by a monotone key, so a point can only be dominated by points earlier in the
// order or with the same key (the topological-sort property of Section 2 that
// SFS relies on, with equal keys tested both ways).
#include "sky_internal.h"
#include "sky_domtest.h"

// Query rows: lane l of row q holds point q * 64 + l of a query group, packed
// so that live points come first; am[q] is the wave mask of row q's lanes
// whose point is still alive. Alive state lives in scalar masks, so the
// tests' compare results (lane masks) combine with it on the scalar unit.
template <int PPL>
__device__ __forceinline__ bool any_live(const uint64_t (&am)[PPL])
{
    uint64_t a = 0;
#pragma unroll
    for (int q = 0; q < PPL; ++q) a |= am[q];
    return a != 0;
}

// Work tickets of a persistent wave. The item space is dealt round-robin to
// SKY_TICK_C classes, each with its own counter in its own 64-byte line
// (same-address atomics serialise, so one shared counter caps the item rate);
// wave w draws from class w % SKY_TICK_C, and inside a class items are handed
// out dynamically. All 64 lanes add 1 (so the call sits in no lane-divergent
// branch): the counter advances by 64 per ticket and the wave's ticket is lane
// 0's old value / 64. These kernels have no workgroup barrier at all.
struct Tickets {
    uint32_t *ctr;
    uint32_t cls;
};

__device__ __forceinline__ Tickets wave_tickets(uint32_t *set)
{
    const uint32_t gw = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t cls = gw % SKY_TICK_C;
    return Tickets{set + cls * 16, cls};
}

// A wave's work counts: lane tests issued, corner checks and lane tests of
// alive query slots. Only the kernels built to count (CNT) keep them; the
// others carry no counters at all, which leaves the scans their scalar
// registers (and no counter in private memory).
template <bool CNT>
struct Work {
    uint64_t rec = 0, blk = 0, alive = 0;
    __device__ __forceinline__ void add_rec(uint64_t v) { rec += v; }
    __device__ __forceinline__ void add_blk(uint64_t v) { blk += v; }
    __device__ __forceinline__ void add_alive(uint64_t v) { alive += v; }
};
template <>
struct Work<false> {
    __device__ __forceinline__ void add_rec(uint64_t) {}
    __device__ __forceinline__ void add_blk(uint64_t) {}
    __device__ __forceinline__ void add_alive(uint64_t) {}
};

template <int PPL>
__device__ __forceinline__ uint32_t live_slots(const uint64_t (&am)[PPL])
{
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < PPL; ++q) c += (uint32_t)__popcll(am[q]);
    return c;
}

// Add a wave's work counts (lane tests issued, corner checks, lane tests of
// alive query slots; wave-uniform) to its class's slots of wcnt
// ([SKY_TICK_C][8] uint64, 64-byte lines).
__device__ __forceinline__ void flush_work(uint64_t *wcnt, uint32_t cls, const Work<true> &wk)
{
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((unsigned long long *)&wcnt[cls * 8], (unsigned long long)(wk.rec * 64));
        atomicAdd((unsigned long long *)&wcnt[cls * 8 + 1], (unsigned long long)(wk.blk * 64));
        atomicAdd((unsigned long long *)&wcnt[cls * 8 + 2], (unsigned long long)wk.alive);
    }
}
__device__ __forceinline__ void flush_work(uint64_t *, uint32_t, const Work<false> &) {}

__device__ __forceinline__ uint64_t next_item(const Tickets &T)
{
    const uint32_t v = atomicAdd(T.ctr, 1u);
    return (uint64_t)(__builtin_amdgcn_readfirstlane(v) >> 6) * SKY_TICK_C + T.cls;
}

// Position of the k-th set bit (k counted from 0, k < popcount) of a 64-bit
// mask that is the same in every lane: a binary search over the popcounts of
// its halves, quarters, ...; branch-free per lane.
__device__ __forceinline__ uint32_t select_bit(uint64_t m, uint32_t k)
{
    uint32_t pos = 0;
    const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
    uint32_t c = (uint32_t)__popc(lo);
    bool up = k >= c;
    k -= up ? c : 0u;
    pos += up ? 32u : 0u;
    uint32_t w = up ? hi : lo;
#pragma unroll
    for (int s = 16; s >= 1; s >>= 1) {
        c = (uint32_t)__popc(w & ((1u << s) - 1u));
        up = k >= c;
        k -= up ? c : 0u;
        pos += up ? (uint32_t)s : 0u;
        w = up ? (w >> s) : w;
    }
    return pos;
}

// Loads the live points of a query group of len <= 64 * PPL records at src,
// packed: the group's points not marked in dead[0 .. len), in their order,
// fill row 0 then row 1 (lane l of row q takes the (64 q + l)-th one). pos[q]
// is the group offset of the lane's point, am[q] the mask of lanes that hold
// one. Returns how many points are live.
template <int DP, int PPL>
__device__ __forceinline__ uint32_t load_live(const uint32_t *__restrict__ src, uint32_t len,
                                              const uint8_t *__restrict__ dead, uint32_t (&x)[PPL][DP - 2],
                                              uint64_t (&K)[PPL], uint64_t (&am)[PPL], uint32_t (&pos)[PPL])
{
    const uint32_t lane = threadIdx.x & 63;
    uint64_t m[PPL];
    uint32_t c[PPL + 1];
    c[0] = 0;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const uint32_t o = q * 64 + lane;
        m[q] = __ballot(o < len && !dead[o < len ? o : 0]);
        c[q + 1] = c[q] + (uint32_t)__popcll(m[q]);
    }
    const uint32_t total = c[PPL];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        const uint32_t rank = r * 64 + lane;
        const bool has = rank < total;
        uint32_t p = 0;
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            if (rank >= c[q] && rank < c[q + 1]) p = q * 64 + select_bit(m[q], rank - c[q]);
        pos[r] = p;
        am[r] = __ballot(has);
        const uint4 *s = reinterpret_cast<const uint4 *>(src + (size_t)(has ? p : 0) * DP);
        uint32_t w[DP];
#pragma unroll
        for (int k = 0; k < DP / 4; ++k) {
            const uint4 v = s[k];
            w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
        }
#pragma unroll
        for (int k = 0; k < DP - 2; ++k) x[r][k] = w[k];
        K[r] = ((uint64_t)w[DP - 1] << 32) | w[DP - 2];
    }
    return total;
}

// Marks dead every packed point that was live before (m0) and is not now (am).
template <int PPL>
__device__ __forceinline__ void store_dead(uint8_t *dead, const uint64_t (&m0)[PPL], const uint64_t (&am)[PPL],
                                           const uint32_t (&pos)[PPL])
{
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < PPL; ++q)
        if (((m0[q] & ~am[q]) >> lane) & 1ull) dead[pos[q]] = 1;
}

// Scan window records src[0..cnt) against the rows. The window is read-only
// for the whole launch and its address is wave-uniform, so the records arrive
// through scalar loads and every comparison takes a scalar operand. Four
// records per batch; the wave stops when no point is alive.
template <int DP, int NC, int PPL, bool CNT>
__device__ __forceinline__ void scan_sgpr(const uint32_t *__restrict__ src, uint32_t cnt,
                                          const uint32_t (&x)[PPL][DP - 2], const uint64_t (&K)[PPL],
                                          uint64_t (&am)[PPL], Work<CNT> &wk)
{
    constexpr int U = 4;
    uint32_t w = 0;
    const uint32_t *p = src;   // record w (immediate offsets for the batch)
    for (; w + U <= cnt; w += U, p += U * DP) {
        wk.add_rec(U * PPL);
        wk.add_alive(U * live_slots<PPL>(am));
        uint32_t r[U][DP];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < DP; ++k) r[u][k] = p[u * DP + k];
#pragma unroll
        for (int u = 0; u < U; ++u) test_rec<DP, NC, PPL>(r[u], x, K, am);
        if (!any_live<PPL>(am)) return;
    }
    wk.add_rec((cnt - w) * PPL);
    wk.add_alive((cnt - w) * live_slots<PPL>(am));
    for (; w < cnt; ++w) {
        uint32_t r[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) r[k] = src[(size_t)w * DP + k];
        test_rec<DP, NC, PPL>(r, x, K, am);
    }
}

// Scan window records [a, e) of src, gated by corners at three levels: for
// every aligned block of SKY_BLK records, bmin holds the coordinate-wise
// minimum of its records with, in the K words, the presort key of its first
// record, followed by the minima of its SKY_NSUB sub-blocks of SKY_SUB records;
// sbc holds the same for every aligned super-block of SKY_SBB blocks. A record
// can dominate point q only if its super-block's, block's and sub-block's
// corners are <= q in every coordinate, so a super-block (then a block, then a
// sub-block) whose corner is below no alive point of the wave is skipped. When
// the window is one key-sorted run starting at record kfrom, a super-block or
// block starting at or after kfrom whose first key exceeds kmax holds no record
// with a key <= kmax, and neither does any later one: the scan stops there.
// Block corners are read four at a time, the sub-block corners of a block that
// passes together; the wave stops when no point is alive.
template <int DP, int NC, int PPL, bool CNT>
__device__ __forceinline__ void scan_blocks(const uint32_t *__restrict__ src, const uint32_t *__restrict__ bmin,
                                            const uint32_t *__restrict__ sbc, uint32_t a, uint32_t e, uint32_t kfrom, uint64_t kmax,
                                            const uint32_t (&x)[PPL][DP - 2], const uint64_t (&K)[PPL],
                                            uint64_t (&am)[PPL], Work<CNT> &wk)
{
    constexpr int ND = DP - 2, V = 4;
    if (a >= e) return;
    const uint32_t be = ((e - 1) >> SKY_BLK_SH) + 1;   // exclusive end block (uniform)
    uint32_t b = a >> SKY_BLK_SH;
    while (b < be) {
        // the super-block of block b: its corner first (and the key stop at its first record)
        const uint32_t sb0 = b - b % SKY_SBB;
        const uint32_t *sc = sbc + (size_t)(sb0 / SKY_SBB) * DP;
        uint32_t cs0[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) cs0[k] = sc[k];
        const uint64_t ks = ((uint64_t)cs0[DP - 1] << 32) | cs0[DP - 2];
        if ((sb0 << SKY_BLK_SH) >= kfrom && ks > kmax) return;   // no record from here on has a key <= kmax
        const uint32_t bend = min(be, sb0 + SKY_SBB);
        wk.add_blk(PPL);
        if (!corner_hits<ND, NC, PPL>(cs0, x, am)) {
            b = bend;
            continue;
        }
        for (uint32_t b0 = b; b0 < bend; b0 += V) {
            wk.add_blk(V * PPL);
            uint32_t c[V][DP];
            const uint32_t *cb = bmin + (size_t)b0 * SKY_CSTRIDE * DP;   // immediate offsets for the batch
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int k = 0; k < DP; ++k) c[v][k] = cb[v * SKY_CSTRIDE * DP + k];
            uint32_t pass = 0, stop = bend;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const uint32_t blk = b0 + v;
                const uint64_t k0 = ((uint64_t)c[v][DP - 1] << 32) | c[v][DP - 2];
                if (blk < stop && (blk << SKY_BLK_SH) >= kfrom && k0 > kmax) stop = blk;   // uniform
                if (blk < stop && corner_hits<ND, NC, PPL>(c[v], x, am)) pass |= 1u << v;
            }
            while (pass) {
                const int v = __builtin_ctz(pass);
                pass &= pass - 1;
                const uint32_t blk = b0 + v;
                const uint32_t *sc2 = bmin + ((size_t)blk * SKY_CSTRIDE + 1) * DP;
                uint32_t cs[SKY_NSUB][ND];
#pragma unroll
                for (int u = 0; u < (int)SKY_NSUB; ++u)
#pragma unroll
                    for (int k = 0; k < ND; ++k) cs[u][k] = sc2[u * DP + k];
                wk.add_blk(SKY_NSUB * PPL);
                uint32_t spass = 0;
#pragma unroll
                for (int u = 0; u < (int)SKY_NSUB; ++u)
                    if (corner_hits<ND, NC, PPL>(cs[u], x, am)) spass |= 1u << u;
                while (spass) {
                    const int u = __builtin_ctz(spass);
                    spass &= spass - 1;
                    const uint32_t s0 = (blk << SKY_BLK_SH) + ((uint32_t)u << SKY_SUB_SH);
                    const uint32_t r0 = max(a, s0), r1 = min(e, s0 + SKY_SUB);
                    if (r0 >= r1) continue;
                    scan_sgpr<DP, NC, PPL, CNT>(src + (size_t)r0 * DP, r1 - r0, x, K, am, wk);
                    if (!any_live<PPL>(am)) return;
                }
            }
            if (stop < bend) return;   // the key stop: no later record has a key <= kmax
        }
        b = bend;
    }
}

// ------------------------------------------------------------------ local skylines
// A point of partition j is in the local skyline u_j iff no point of r_j'
// dominates it -- the set SFS computes (Algorithm 1). The records are sorted
// by a monotone key, so a dominator of a point comes earlier or carries the
// same key (the run rule): the scan covers every earlier record, the point's
// own query group, and the rest of the equal-key run that ends the group.
// Query groups: 64*PPL consecutive points of one partition, numbered
// partition-major (group g of partition j = gpart[g] is st_off[j] + c). Items:
// for group g with window length c*B (all earlier points of its partition),
// segments s = 0..nseg-1 of S records, then s = nseg, the group's own records
// and the run after it. Items run segment-major (s outermost), so the
// strongest points of every partition are tested first; a killed point is
// recorded in dead[] and skipped by items that load it later: an item loads
// only the group's live points, packed into the fewest rows of 64 query slots
// that hold them, and tests window records against those rows only. No item
// waits for another.
__device__ __forceinline__ uint32_t seg_len(uint32_t maxc, uint32_t B, uint32_t smin)
{
    uint32_t S = (maxc * B / 64 + 63) & ~63u;   // at most ~65 items per group
    return S < smin ? smin : S;
}

// The window scan of one local item with R rows of query slots.
template <int DP, int NC, int R, bool CNT>
__device__ __forceinline__ void local_item_scan(const uint32_t *__restrict__ raw, const uint64_t *__restrict__ key,
                                                const uint32_t *__restrict__ bmin, const uint32_t *__restrict__ sbc,
                                                uint32_t sidx, uint32_t nseg,
                                                uint32_t S, uint32_t pbeg, uint32_t pend, uint32_t qstart,
                                                uint32_t qlen, const uint32_t (&x)[R][DP - 2],
                                                const uint64_t (&K)[R], uint64_t (&am)[R], Work<CNT> &wk)
{
    if (sidx < nseg) {
        const uint32_t a = pbeg + sidx * S, e = min(pbeg + (sidx + 1) * S, qstart);
        scan_blocks<DP, NC, R, CNT>(raw, bmin, sbc, a, e, 0xFFFFFFFFu, ~0ull, x, K, am, wk);
    } else {
        // the group's own records, every pair (equal keys may dominate either
        // way; a record never dominates itself or its duplicates: equal K),
        // then the records after the group that share its last key
        scan_sgpr<DP, NC, R, CNT>(raw + (size_t)qstart * DP, qlen, x, K, am, wk);
        const uint32_t qend = qstart + qlen;
        const uint64_t klast = key[qend - 1];
        uint32_t we = qend;
        while (we < pend && key[we] == klast) ++we;
        we = __builtin_amdgcn_readfirstlane(we);
        if (we > qend && any_live<R>(am))
            scan_sgpr<DP, NC, R, CNT>(raw + (size_t)qend * DP, we - qend, x, K, am, wk);
    }
}

// The scan of a local item on its first R rows (the rows that hold live points).
template <int DP, int NC, int PPL, int R, bool CNT>
__device__ __forceinline__ void local_rows(const uint32_t *__restrict__ raw, const uint64_t *__restrict__ key,
                                           const uint32_t *__restrict__ bmin, const uint32_t *__restrict__ sbc,
                                           uint32_t sidx, uint32_t nseg,
                                           uint32_t S, uint32_t pbeg, uint32_t pend, uint32_t qstart, uint32_t qlen,
                                           const uint32_t (&x)[PPL][DP - 2], const uint64_t (&K)[PPL],
                                           uint64_t (&am)[PPL], Work<CNT> &wk)
{
    uint32_t xr[R][DP - 2];
    uint64_t Kr[R], ar[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int k = 0; k < DP - 2; ++k) xr[r][k] = x[r][k];
        Kr[r] = K[r];
        ar[r] = am[r];
    }
    local_item_scan<DP, NC, R, CNT>(raw, key, bmin, sbc, sidx, nseg, S, pbeg, pend, qstart, qlen, xr, Kr, ar, wk);
#pragma unroll
    for (int r = 0; r < R; ++r) am[r] = ar[r];
}

// CAP (records of at most 8 words): the kernel is held to 64 VGPRs, so 8 waves
// fit per SIMD. That measured faster than 6 waves on inputs up to a few
// million points, and slower on larger ones.
template <int DP, int NC, int PPL, bool CAP, bool CNT>
__global__ __launch_bounds__(256, CAP ? 8 : 1) void k_local_items(const uint32_t *__restrict__ raw,
                                                    const uint64_t *__restrict__ key,
                                                    const uint32_t *__restrict__ poff,
                                                    const uint32_t *__restrict__ bmin,
                                                    const uint32_t *__restrict__ sbc,
                                                    const uint32_t *__restrict__ st_off,
                                                    const uint32_t *__restrict__ gpart,
                                                    const uint32_t *__restrict__ xlist, uint32_t smin,
                                                    uint32_t *ctrl, uint32_t *tick, uint8_t *dead, uint64_t *wcnt)
{
    constexpr int B = 64 * PPL, ND = DP - 2;
    const uint32_t G = __builtin_amdgcn_readfirstlane(ctrl[C_NCHUNK]);
    const uint32_t maxc = __builtin_amdgcn_readfirstlane(ctrl[C_MAXC]);
    if (G == 0) return;
    const uint32_t S = seg_len(maxc, B, smin);
    const uint32_t rounds = (maxc ? (maxc - 1) * B + S - 1 : 0) / S + 1;   // max items per group
    // Queues: with xlist, one per XCD holding the items of its partitions (the
    // window records then stay in that XCD's L2); a wave drains its own XCD's
    // queue first, then the others'. Without, a single queue. Each queue is
    // dealt over QC ticket classes.
    const uint32_t NQ = xlist ? SKY_NXCD : 1, QC = SKY_TICK_C / NQ;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t x0 = xlist ? blockIdx.x % SKY_NXCD : 0;
    const uint32_t cl = xlist ? ((blockIdx.x / SKY_NXCD) * (blockDim.x >> 6) + wv) % QC
                              : (blockIdx.x * (blockDim.x >> 6) + wv) % QC;
    Work<CNT> wk;
    for (uint32_t qi = 0; qi < NQ; ++qi) {
      const uint32_t xq = (x0 + qi) % NQ;
      uint32_t Gq = G, qbase = 0;
      if (xlist) {
          Gq = __builtin_amdgcn_readfirstlane(ctrl[C_XG0 + xq]);
          for (uint32_t y = 0; y < xq; ++y) qbase += __builtin_amdgcn_readfirstlane(ctrl[C_XG0 + y]);
      }
      // rounds <= 65 and Gq <= n / 64, so the item count fits 32 bits
      const uint32_t total = rounds * Gq;
      uint32_t *ctr = tick + (xq * QC + cl) * 16;
      for (;;) {
        const uint32_t t = (__builtin_amdgcn_readfirstlane(atomicAdd(ctr, 1u)) >> 6) * QC + cl;
        if (t >= total) break;
        const uint32_t sidx = t / Gq, gi = t - sidx * Gq;
        const uint32_t g = xlist ? __builtin_amdgcn_readfirstlane(xlist[qbase + gi]) : gi;
        const uint32_t j = __builtin_amdgcn_readfirstlane(gpart[g]);
        const uint32_t c = g - __builtin_amdgcn_readfirstlane(st_off[j]);
        const uint32_t wlen = c * B, nseg = (wlen + S - 1) / S;
        if (sidx > nseg) continue;
        const uint32_t pbeg = __builtin_amdgcn_readfirstlane(poff[j]);
        const uint32_t pend = __builtin_amdgcn_readfirstlane(poff[j + 1]);
        const uint32_t qstart = pbeg + c * B, qlen = min((uint32_t)B, pend - qstart);
        uint32_t x[PPL][ND], pos[PPL];
        uint64_t K[PPL], am[PPL], m0[PPL];
        const uint32_t live = load_live<DP, PPL>(raw + (size_t)qstart * DP, qlen, dead + qstart, x, K, am, pos);
        if (live == 0) continue;
#pragma unroll
        for (int q = 0; q < PPL; ++q) m0[q] = am[q];
        const uint32_t rows = (live + 63) >> 6;   // rows that hold the live points
        if (rows == 1)
            local_rows<DP, NC, PPL, 1, CNT>(raw, key, bmin, sbc, sidx, nseg, S, pbeg, pend, qstart, qlen, x, K, am, wk);
        else if (PPL >= 4 && rows == 2)
            local_rows<DP, NC, PPL, (PPL >= 4 ? 2 : 1), CNT>(raw, key, bmin, sbc, sidx, nseg, S, pbeg, pend, qstart, qlen, x,
                                                        K, am, wk);
        else if (PPL >= 4 && rows == 3)
            local_rows<DP, NC, PPL, (PPL >= 4 ? 3 : 1), CNT>(raw, key, bmin, sbc, sidx, nseg, S, pbeg, pend, qstart, qlen, x,
                                                        K, am, wk);
        else
            local_rows<DP, NC, PPL, PPL, CNT>(raw, key, bmin, sbc, sidx, nseg, S, pbeg, pend, qstart, qlen, x, K, am, wk);
        store_dead<PPL>(dead + qstart, m0, am, pos);
      }
    }
    flush_work(wcnt, (x0 * QC + cl) % SKY_TICK_C, wk);
}

template <int PPL, bool CAP>
static hipError_t local_items_ppl(int DP, int NC, uint32_t smin, const uint32_t *raw, const uint64_t *key,
                                  const uint32_t *poff, const uint32_t *bmin, const uint32_t *sbc,
                                  const uint32_t *st_off,
                                  const uint32_t *gpart, const uint32_t *xlist, uint32_t *ctrl, uint32_t *tick,
                                  uint8_t *dead, uint64_t *wcnt, int n_wg, hipStream_t s)
{
#define L_CASE(X, C)                                                                                           \
    case X * 32 + C:                                                                                           \
        if (wcnt)                                                                                              \
            hipLaunchKernelGGL((k_local_items<X, C, PPL, CAP && X <= 8, true>), dim3(n_wg), dim3(256), 0, s, raw,  \
                               key, poff, bmin, sbc, st_off, gpart, xlist, smin, ctrl, tick, dead, wcnt);       \
        else                                                                                                   \
            hipLaunchKernelGGL((k_local_items<X, C, PPL, CAP && X <= 8, false>), dim3(n_wg), dim3(256), 0, s, raw, \
                               key, poff, bmin, sbc, st_off, gpart, xlist, smin, ctrl, tick, dead, wcnt);       \
        break;
    switch (DP * 32 + NC) {
        L_CASE(4, 2) L_CASE(8, 4) L_CASE(8, 6) L_CASE(12, 8) L_CASE(12, 10) L_CASE(16, 12) L_CASE(16, 14)
        L_CASE(20, 16)
        default: return hipErrorInvalidValue;
    }
#undef L_CASE
    return hipGetLastError();
}

// ppl: query points per lane (a query group is 64 * ppl points; the chunk
// table must use the same group size); smin: smallest window segment; n_in:
// the call's input size, which picks the register-bounded kernel for inputs
// of at most SKY_LOCAL_CAP_N points.
#define SKY_LOCAL_CAP_N (4u << 20)
hipError_t launch_local_sky(int d, int ppl, uint32_t smin, const uint32_t *raw, const uint64_t *key,
                            const uint32_t *poff, const uint32_t *bmin, const uint32_t *st_off,
                            const uint32_t *gpart, const uint32_t *xlist, uint32_t *ctrl, uint32_t *tick,
                            uint8_t *dead, uint64_t *wcnt, int n_wg, uint32_t n_in, hipStream_t s)
{
    const int DP = sky_dp(d), NC = sky_nc(d);
    const bool cap = n_in <= SKY_LOCAL_CAP_N;
    const uint32_t *sbc = bmin + sky_block_corner_words(n_in, DP);   // the super-block corners
#define P_CASE(PP, C)                                                                                         \
    return local_items_ppl<PP, C>(DP, NC, smin, raw, key, poff, bmin, sbc, st_off, gpart, xlist, ctrl, tick,   \
                                  dead, wcnt, n_wg, s)
    if (ppl == 4) P_CASE(4, false);
    if (ppl == 2) {
        if (cap) P_CASE(2, true);
        P_CASE(2, false);
    }
    if (ppl == 1) {
        if (cap) P_CASE(1, true);
        P_CASE(1, false);
    }
#undef P_CASE
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ block lower corners
// Corner records of every block of SKY_BLK records of rec[0..*n_dev): first
// the block's (coordinate-wise minimum of its records, the presort key of its
// first record in the K words), then one per sub-block of SKY_SUB records
// (minimum, K words 0). A partial block takes the minimum of what it holds; a
// sub-block with no record gets all-ones, which passes no corner test. Then
// one per super-block of SKY_SBB blocks in sbc (minimum, the presort key of
// its first record). One workgroup per super-block, of at most 16 waves that
// take SKY_SBB / 16 consecutive blocks each, one record per lane.
#define BM_WAVES (SKY_SBB < 16 ? SKY_SBB : 16)
#define BM_WG (BM_WAVES * 64)
template <int DP>
__global__ __launch_bounds__(BM_WG) void k_block_min(const uint32_t *__restrict__ rec,
                                                     const uint64_t *__restrict__ key, const uint32_t *n_dev,
                                                     uint32_t *__restrict__ bmin, uint32_t *__restrict__ sbc)
{
    static_assert(SKY_BLK == 64 && SKY_SUB <= 32, "one record per lane; sub-blocks of SKY_SUB lanes");
    constexpr int ND = DP - 2, BPW = SKY_SBB / BM_WAVES;   // blocks per wave
    __shared__ uint32_t s_m[BM_WAVES][ND];
    const uint32_t n = *n_dev;
    const uint32_t nb = (n + SKY_BLK - 1) >> SKY_BLK_SH;
    const uint32_t nsb = (nb + SKY_SBB - 1) / SKY_SBB;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (uint32_t sbk = blockIdx.x; sbk < nsb; sbk += gridDim.x) {   // uniform per workgroup
        uint32_t sm[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) sm[k] = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const uint32_t b = sbk * SKY_SBB + wv * BPW + i;
            if (b < nb) {   // wave-uniform
                uint32_t m[ND];
#pragma unroll
                for (int k = 0; k < ND; ++k) m[k] = 0xFFFFFFFFu;
                const uint32_t r = (b << SKY_BLK_SH) + lane;
                if (r < n) {
                    const uint4 *src = reinterpret_cast<const uint4 *>(rec + (size_t)r * DP);
#pragma unroll
                    for (int k4 = 0; k4 < DP / 4; ++k4) {
                        const uint4 v = src[k4];
                        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            if (4 * k4 + t < ND) m[4 * k4 + t] = w[t];
                    }
                }
                // sub-block minima (16-lane groups), then the block's
#pragma unroll
                for (int k = 0; k < ND; ++k)
                    for (int o = 1; o < (int)SKY_SUB; o <<= 1) m[k] = min(m[k], (uint32_t)__shfl_xor((int)m[k], o, 64));
                uint32_t *cb = bmin + (size_t)b * SKY_CSTRIDE * DP;
                if ((lane & (SKY_SUB - 1)) == 0) {
                    uint32_t *cs = cb + (size_t)(1 + (lane >> SKY_SUB_SH)) * DP;
#pragma unroll
                    for (int k = 0; k < ND; ++k) cs[k] = m[k];
                    cs[DP - 2] = 0;
                    cs[DP - 1] = 0;
                }
#pragma unroll
                for (int k = 0; k < ND; ++k)
                    for (int o = SKY_SUB; o < 64; o <<= 1) m[k] = min(m[k], (uint32_t)__shfl_xor((int)m[k], o, 64));
                const uint64_t k0 = key[(size_t)b << SKY_BLK_SH];
                uint32_t out = lane == (uint32_t)(DP - 2) ? (uint32_t)k0 : (uint32_t)(k0 >> 32);
#pragma unroll
                for (int k = 0; k < ND; ++k)
                    if (lane == (uint32_t)k) out = m[k];
                if (lane < (uint32_t)DP) cb[lane] = out;
#pragma unroll
                for (int k = 0; k < ND; ++k) sm[k] = min(sm[k], m[k]);
            }
        }
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < ND; ++k) s_m[wv][k] = sm[k];
        __syncthreads();
        if (threadIdx.x < (uint32_t)DP) {
            const uint32_t k = threadIdx.x;
            uint32_t v;
            if (k < (uint32_t)ND) {
                v = s_m[0][k];
                for (int w = 1; w < BM_WAVES; ++w) v = min(v, s_m[w][k]);
            } else {
                const uint64_t k0 = key[(size_t)sbk * SKY_SBB << SKY_BLK_SH];
                v = k == (uint32_t)(DP - 2) ? (uint32_t)k0 : (uint32_t)(k0 >> 32);
            }
            sbc[(size_t)sbk * DP + k] = v;
        }
        __syncthreads();
    }
}

hipError_t launch_block_min(int d, const uint32_t *rec, const uint64_t *key, const uint32_t *n_dev, uint32_t n_max,
                            uint32_t *bmin, hipStream_t s)
{
    const uint32_t nb = (n_max + SKY_BLK - 1) >> SKY_BLK_SH;
    uint32_t blocks = (nb + SKY_SBB - 1) / SKY_SBB;   // one workgroup per super-block
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    const int DP = sky_dp(d);
    uint32_t *sbc = bmin + sky_block_corner_words(n_max, DP);
#define B_CASE(X)                                                                                           \
    case X:                                                                                                 \
        hipLaunchKernelGGL(k_block_min<X>, dim3(blocks), dim3(BM_WG), 0, s, rec, key, n_dev, bmin, sbc);   \
        break;
    switch (DP) {
        B_CASE(4) B_CASE(8) B_CASE(12) B_CASE(16) B_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef B_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------ union of local skylines
// u = the points never marked dead, compacted stably (so each u_j stays in
// presort order) into dense records, ids and keys; upoff[j] = |u_0| +
// ... + |u_{j-1}|. Two passes over segments of seg sorted positions (at least
// UN_SEG, at most 1024 segments): the write pass sums the counts of the
// segments before its own, so no scan launch sits between them.
#define UN_SEG 4096

// The sum of one value per thread over a 256-thread workgroup, returned to
// every thread (s_tmp: 4 words of LDS).
__device__ __forceinline__ uint32_t block_sum256(uint32_t v, uint32_t *s_tmp)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
    __syncthreads();
    const uint32_t r = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(SKY_WG) void k_union_count(const uint8_t *__restrict__ dead, const uint32_t *n_dev,
                                                       uint32_t seg, uint32_t *wg_cnt)
{
    __shared__ uint32_t s_c;
    const uint32_t n = *n_dev;
    if (threadIdx.x == 0) s_c = 0;
    __syncthreads();
    const uint32_t b0 = blockIdx.x * seg, e0 = min(n, b0 + seg);
    uint32_t c = 0;
    for (uint32_t r = b0 + threadIdx.x; r < e0; r += SKY_WG) c += dead[r] ? 0u : 1u;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_c, c);
    __syncthreads();
    if (threadIdx.x == 0) wg_cnt[blockIdx.x] = s_c;
}

template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_union_write(const uint8_t *__restrict__ dead, const uint32_t *n_dev,
                                                       uint32_t seg, const uint32_t *__restrict__ wg_cnt,
                                                       const uint32_t *__restrict__ rec,
                                                       const uint32_t *__restrict__ sid,
                                                       const uint64_t *__restrict__ skey, uint32_t *urank,
                                                       uint32_t *__restrict__ urec, uint32_t *__restrict__ uid,
                                                       uint64_t *__restrict__ ukey, uint32_t *ctrl)
{
    __shared__ uint32_t s_w[4];
    const uint32_t n = *n_dev;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t b0 = blockIdx.x * seg, e0 = min(n, b0 + seg);
    // this segment's first position in u: the survivors of the segments before it
    uint32_t before = 0;
    for (uint32_t j = threadIdx.x; j < blockIdx.x; j += SKY_WG) before += wg_cnt[j];
    uint32_t pos = block_sum256(before, s_w);
    for (uint32_t base = b0; base < b0 + seg; base += SKY_WG) {
        const uint32_t r = base + threadIdx.x;
        const bool a = r < e0 && !dead[r];
        const uint64_t m = __ballot(a);
        if (lane == 0) s_w[wv] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t off = pos, tot = 0;
        for (uint32_t w = 0; w < 4; ++w) {
            if (w < wv) off += s_w[w];
            tot += s_w[w];
        }
        off += (uint32_t)__popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull));
        if (r < e0) urank[r] = off;    // rank among alive positions before r (exclusive)
        if (a) {
            const uint4 *src = reinterpret_cast<const uint4 *>(rec + (size_t)r * DP);
            uint4 *dst = reinterpret_cast<uint4 *>(urec + (size_t)off * DP);
#pragma unroll
            for (int k = 0; k < DP / 4; ++k) dst[k] = src[k];
            uid[off] = sid[r];
            ukey[off] = skey[r];
        }
        pos += tot;
        __syncthreads();
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) ctrl[C_NU] = pos;   // the size of u
}

__global__ __launch_bounds__(1024) void k_union_offsets(const uint32_t *__restrict__ poff, int np,
                                                        const uint32_t *__restrict__ urank, const uint32_t *n_dev,
                                                        uint32_t *upoff, uint32_t *ctrl, int64_t *local_sizes)
{
    __shared__ uint32_t s_m[16];
    const uint32_t n = *n_dev, nu = ctrl[C_NU];
    for (int j = threadIdx.x; j <= np; j += 1024) {
        const uint32_t pj = poff[j];
        upoff[j] = pj < n ? urank[pj] : nu;
    }
    __syncthreads();
    uint32_t mx = 0;
    for (int j = threadIdx.x; j < np; j += 1024) {
        const uint32_t sz = upoff[j + 1] - upoff[j];
        mx = max(mx, sz);
        if (local_sizes) local_sizes[j] = (int64_t)sz;
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0;
        for (int w = 0; w < 16; ++w) m = max(m, s_m[w]);
        ctrl[C_MAXU] = m;
    }
}

hipError_t launch_union(int d, const uint8_t *dead, const uint32_t *n_dev, uint32_t n_max, const uint32_t *rec,
                        const uint32_t *sid, const uint64_t *skey, const uint32_t *poff, int np, uint32_t *wg_cnt,
                        uint32_t *urank, uint32_t *urec, uint32_t *uid, uint64_t *ukey, uint32_t *upoff,
                        uint32_t *ctrl, int64_t *local_sizes, hipStream_t s, bool offsets)
{
    uint32_t seg = (n_max + 1023) / 1024;   // at most 1024 segments
    seg = seg < UN_SEG ? UN_SEG : (seg + SKY_WG - 1) / SKY_WG * SKY_WG;
    const uint32_t nwg = n_max > 0 ? (n_max + seg - 1) / seg : 1;
    hipLaunchKernelGGL(k_union_count, dim3(nwg), dim3(SKY_WG), 0, s, dead, n_dev, seg, wg_cnt);
    const int DP = sky_dp(d);
#define U_CASE(X)                                                                                                    \
    case X:                                                                                                          \
        hipLaunchKernelGGL(k_union_write<X>, dim3(nwg), dim3(SKY_WG), 0, s, dead, n_dev, seg, wg_cnt, rec, sid, skey, \
                           urank, urec, uid, ukey, ctrl);                                                            \
        break;
    switch (DP) {
        U_CASE(4) U_CASE(8) U_CASE(12) U_CASE(16) U_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef U_CASE
    if (offsets)   // else the chunk table's launch derives them (UnionOffsets)
        hipLaunchKernelGGL(k_union_offsets, dim3(1), dim3(1024), 0, s, poff, np, urank, n_dev, upoff, ctrl,
                           local_sizes);
    return hipGetLastError();
}

// ------------------------------------------------------------------ NoSeq merge
// Sky(r) = union_i Sky_{pd_i}(u_i) (Proposition 2): every point of u_i is
// tested against its partition's potential dominators pd_i, and survives iff
// none dominates it. pd_i: Sliced u_j, j < i; Grid u_j with c_j <= c_i in
// every dimension, j != i (the weak grid-dominance superset, always sound);
// Angular every u_j, j != i. Only points with a presort key no larger than
// the dominated point's can dominate, and u_j is sorted by that key, so u_j is
// scanned only up to the largest key of the query group (inclusive).
// Items: (candidate index, segment of mseg records of u_j, query group of
// 64*PPL points of one u_i), the candidate index outermost; for Sliced the
// candidates run from the nearest lower slice downwards. With ppi < np the
// partitions are ppi slices of each of several independent instances, and a
// query's candidates are the earlier slices of its own instance. A query point killed
// by any item is marked dead, and items that load it later skip it.
__device__ __forceinline__ bool grid_weakly_below(uint32_t j, uint32_t i, const GridSpec &g)
{
    for (int k = 0; k < g.d; ++k) {
        const uint32_t m = (uint32_t)g.m[k];
        if (j % m > i % m) return false;
        j /= m;
        i /= m;
    }
    return true;
}

// The block scan of a merge item on its first R rows.
template <int DP, int NC, int PPL, int R, bool CNT>
__device__ __forceinline__ void merge_rows(const uint32_t *__restrict__ urec, const uint32_t *__restrict__ ubmin,
                                           const uint32_t *__restrict__ ubc, uint32_t a, uint32_t e, uint32_t kfrom, uint64_t kmax,
                                           const uint32_t (&x)[PPL][DP - 2], const uint64_t (&K)[PPL],
                                           uint64_t (&am)[PPL], Work<CNT> &wk)
{
    uint32_t xr[R][DP - 2];
    uint64_t Kr[R], ar[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int k = 0; k < DP - 2; ++k) xr[r][k] = x[r][k];
        Kr[r] = K[r];
        ar[r] = am[r];
    }
    scan_blocks<DP, NC, R, CNT>(urec, ubmin, ubc, a, e, kfrom, kmax, xr, Kr, ar, wk);
#pragma unroll
    for (int r = 0; r < R; ++r) am[r] = ar[r];
}

template <int DP, int NC, int PPL, bool CNT>
__global__ __launch_bounds__(256) void k_merge_items(const uint32_t *__restrict__ urec,
                                                    const uint32_t *__restrict__ ubmin,
                                                    const uint32_t *__restrict__ ubc,
                                                    const uint64_t *__restrict__ ukey,
                                                    const uint32_t *__restrict__ upoff,
                                                    const uint32_t *__restrict__ st_off,
                                                    const uint32_t *__restrict__ gpart, int np, int ppi,
                                                    int part_kind, GridSpec pg, uint32_t mseg, uint32_t *ctrl,
                                                    uint32_t *tick, uint8_t *udead, uint64_t *wcnt)
{
    constexpr int B = 64 * PPL, ND = DP - 2;
    const uint32_t G = __builtin_amdgcn_readfirstlane(ctrl[C_NCHUNK2]);
    const uint32_t maxu = __builtin_amdgcn_readfirstlane(ctrl[C_MAXU]);
    const uint32_t nu = __builtin_amdgcn_readfirstlane(ctrl[C_NU]);
    const uint32_t nsm = (maxu + mseg - 1) / mseg;
    const uint64_t per_j = (uint64_t)nsm * G;
    // Two item spaces. Per candidate partition: (j, segment of u_j, group), whose
    // scans stop at the group's largest key. Over one range: (segment, group) of
    // the contiguous candidate range -- Sliced: all earlier slices, u[upoff[0],
    // upoff[i]); Angular, Random, none: all of u (a point's own u_i never
    // dominates it, so scanning it too is harmless). Many small partitions make
    // the first space about p^2 mostly empty items, while the range form scans
    // about twice the records (no key stop). Per group, the first costs
    // nsm * p tickets plus half of the range's records; the range form is taken
    // when its saved tickets, at TICKET_RECS records each (measured: a ticket
    // costs between 4 and 43 record scans), outweigh that (single instance only).
    const uint64_t total_j = per_j * (uint32_t)ppi;   // candidates lie in the query's own instance
    const uint32_t nsr = (nu + mseg - 1) / mseg;
    // Sliced halves both forms' records (only earlier slices): its weight doubles
    const uint64_t TICKET_RECS = part_kind == P_SLICED ? 48 : 24;
    const uint64_t tj = (uint64_t)nsm * (uint32_t)np;
    const bool range = ppi == np && part_kind != P_GRID && tj > nsr && TICKET_RECS * (tj - nsr) > nu;
    const uint64_t total = range ? (uint64_t)nsr * G : total_j;
    const Tickets T = wave_tickets(tick);
    Work<CNT> wk;
    const bool small = total <= 0xFFFFFFFFull;   // 32-bit item arithmetic (uniform)
    for (;;) {
        const uint64_t t = next_item(T);
        if (t >= total) break;
        uint32_t g, a, e, lo0;
        if (range) {
            const uint32_t sg = small ? (uint32_t)t / G : (uint32_t)(t / G);
            g = (uint32_t)t - sg * G;
            const uint32_t i = __builtin_amdgcn_readfirstlane(gpart[g]);
            const uint32_t hi = part_kind == P_SLICED ? __builtin_amdgcn_readfirstlane(upoff[i]) : nu;
            a = sg * mseg;
            if (a >= hi) continue;
            e = min(hi, a + mseg);
            lo0 = 0xFFFFFFFFu;   // several key-sorted runs: no stop at the largest key
        } else {
            uint32_t jidx, sg;
            if (small) {
                const uint32_t t32 = (uint32_t)t, pj = (uint32_t)per_j;
                jidx = t32 / pj;
                const uint32_t rem = t32 - jidx * pj;
                sg = rem / G;
                g = rem - sg * G;
            } else {
                jidx = (uint32_t)(t / per_j);
                const uint64_t rem = t - (uint64_t)jidx * per_j;
                sg = (uint32_t)(rem / G);
                g = (uint32_t)(rem - (uint64_t)sg * G);
            }
            const uint32_t i = __builtin_amdgcn_readfirstlane(gpart[g]);
            uint32_t j;
            bool pd;
            if (part_kind == P_SLICED) {
                pd = jidx < i % (uint32_t)ppi;   // an earlier slice of the same instance
                j = i - 1 - jidx;
            } else {
                j = jidx;
                pd = j != i && (part_kind != P_GRID || grid_weakly_below(j, i, pg));
            }
            if (!pd) continue;
            lo0 = __builtin_amdgcn_readfirstlane(upoff[j]);
            const uint32_t hi0 = __builtin_amdgcn_readfirstlane(upoff[j + 1]);
            a = lo0 + sg * mseg;
            if (a >= hi0) continue;
            e = min(hi0, a + mseg);
        }
        const uint32_t i = __builtin_amdgcn_readfirstlane(gpart[g]);
        const uint32_t c = g - __builtin_amdgcn_readfirstlane(st_off[i]);
        const uint32_t qstart = __builtin_amdgcn_readfirstlane(upoff[i]) + c * B;
        const uint32_t qlen = min((uint32_t)B, __builtin_amdgcn_readfirstlane(upoff[i + 1]) - qstart);
        // largest presort key among the group (the group is key-sorted)
        const uint64_t kmax = ukey[qstart + qlen - 1];
        if (!range && ukey[a] > kmax) continue;   // u_j is key-sorted: nothing from a on can dominate
        uint32_t x[PPL][ND], pos[PPL];
        uint64_t K[PPL], am[PPL], m0[PPL];
        const uint32_t live = load_live<DP, PPL>(urec + (size_t)qstart * DP, qlen, udead + qstart, x, K, am, pos);
        if (live == 0) continue;
#pragma unroll
        for (int q = 0; q < PPL; ++q) m0[q] = am[q];
        const uint32_t rows = (live + 63) >> 6;   // rows that hold the live points
        if (rows == 1)
            merge_rows<DP, NC, PPL, 1, CNT>(urec, ubmin, ubc, a, e, lo0, kmax, x, K, am, wk);
        else if (PPL >= 4 && rows == 2)
            merge_rows<DP, NC, PPL, (PPL >= 4 ? 2 : 1), CNT>(urec, ubmin, ubc, a, e, lo0, kmax, x, K, am, wk);
        else if (PPL >= 4 && rows == 3)
            merge_rows<DP, NC, PPL, (PPL >= 4 ? 3 : 1), CNT>(urec, ubmin, ubc, a, e, lo0, kmax, x, K, am, wk);
        else
            merge_rows<DP, NC, PPL, PPL, CNT>(urec, ubmin, ubc, a, e, lo0, kmax, x, K, am, wk);
        store_dead<PPL>(udead + qstart, m0, am, pos);
    }
    flush_work(wcnt, T.cls, wk);
}

__global__ __launch_bounds__(SKY_WG) void k_mark_alive(const uint8_t *__restrict__ dead,
                                                      const uint32_t *__restrict__ ids, const uint32_t *n_dev,
                                                      uint32_t *skybits)
{
    const uint32_t n = *n_dev;
    for (uint32_t r = blockIdx.x * SKY_WG + threadIdx.x; r < n; r += gridDim.x * SKY_WG)
        if (!dead[r]) {
            const uint32_t id = ids[r];
            atomicOr(&skybits[id >> 5], 1u << (id & 31));
        }
}

hipError_t launch_mark_alive(const uint8_t *dead, const uint32_t *ids, const uint32_t *n_dev, uint32_t n_max,
                             uint32_t *skybits, hipStream_t s)
{
    uint32_t blocks = (n_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_mark_alive, dim3(blocks), dim3(SKY_WG), 0, s, dead, ids, n_dev, skybits);
    return hipGetLastError();
}

template <int PPL>
static hipError_t merge_items_ppl(int DP, int NC, uint32_t mseg, const uint32_t *urec, const uint32_t *ubmin,
                                  const uint32_t *ubc, const uint64_t *ukey, const uint32_t *upoff, const uint32_t *st_off,
                                  const uint32_t *gpart, int np, int ppi, int part_kind, const GridSpec &pg,
                                  uint32_t *ctrl, uint32_t *tick, uint8_t *udead, uint64_t *wcnt, int n_wg,
                                  hipStream_t s)
{
#define M_CASE(X, C)                                                                                          \
    case X * 32 + C:                                                                                          \
        if (wcnt)                                                                                             \
            hipLaunchKernelGGL((k_merge_items<X, C, PPL, true>), dim3(n_wg), dim3(256), 0, s, urec, ubmin, ubc, \
                               ukey, upoff, st_off, gpart, np, ppi, part_kind, pg, mseg, ctrl, tick, udead, wcnt);  \
        else                                                                                                  \
            hipLaunchKernelGGL((k_merge_items<X, C, PPL, false>), dim3(n_wg), dim3(256), 0, s, urec, ubmin, ubc, \
                               ukey, upoff, st_off, gpart, np, ppi, part_kind, pg, mseg, ctrl, tick, udead, wcnt);  \
        break;
    switch (DP * 32 + NC) {
        M_CASE(4, 2) M_CASE(8, 4) M_CASE(8, 6) M_CASE(12, 8) M_CASE(12, 10) M_CASE(16, 12) M_CASE(16, 14)
        M_CASE(20, 16)
        default: return hipErrorInvalidValue;
    }
#undef M_CASE
    return hipGetLastError();
}

// ppl: query points per lane (the chunk table over u must use groups of
// 64 * ppl); mseg: records of u_j per item.
hipError_t launch_merge_noseq(int d, int ppl, uint32_t mseg, const uint32_t *urec, const uint32_t *ubmin,
                              const uint64_t *ukey, const uint32_t *uid, const uint32_t *upoff,
                              const uint32_t *st_off, const uint32_t *gpart, int np, int ppi, int part_kind,
                              const GridSpec &pg, uint32_t *ctrl, uint32_t *tick, uint8_t *udead, uint64_t *wcnt,
                              uint32_t *skybits, uint32_t n_max, int n_wg, hipStream_t s)
{
    const int DP = sky_dp(d), NC = sky_nc(d);
    const uint32_t *ubc = ubmin + sky_block_corner_words(n_max, DP);   // the super-block corners
    if (ppl == 4)
        return merge_items_ppl<4>(DP, NC, mseg, urec, ubmin, ubc, ukey, upoff, st_off, gpart, np, ppi, part_kind, pg, ctrl,
                                  tick, udead, wcnt, n_wg, s);
    if (ppl == 2)
        return merge_items_ppl<2>(DP, NC, mseg, urec, ubmin, ubc, ukey, upoff, st_off, gpart, np, ppi, part_kind, pg, ctrl,
                                  tick, udead, wcnt, n_wg, s);
    if (ppl == 1)
        return merge_items_ppl<1>(DP, NC, mseg, urec, ubmin, ubc, ukey, upoff, st_off, gpart, np, ppi, part_kind, pg, ctrl,
                                  tick, udead, wcnt, n_wg, s);
    return hipErrorInvalidValue;
}

// Built-in work splits: two query points per lane while a record fits in 8
// words, 1024-record segments, 8 workgroups (32 waves) per compute unit.
TuneParams tune_builtin(int d)
{
    const int ppl = sky_dp(d) <= 8 ? 2 : 1;
    return TuneParams{ppl, 1024, ppl, 1024, 8};
}

static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

bool tune_valid(const TuneParams &t)
{
    return (t.lppl == 1 || t.lppl == 2 || t.lppl == 4) && (t.mppl == 1 || t.mppl == 2 || t.mppl == 4) && pow2_in(t.lseg, 256, 8192) &&
           pow2_in(t.mseg, 256, 8192) && t.wgcu >= 1 && t.wgcu <= 8;
}

// Global merge (the final round of Algorithm 2, Sky(u) by SFS): u is re-sorted
// by its presort key and run through the local-skyline kernel as one partition.
__global__ __launch_bounds__(SKY_WG) void k_u_sort_prep(const uint64_t *__restrict__ ukey, const uint32_t *n_dev,
                                                       uint64_t *keys, uint32_t *vals)
{
    const uint32_t n = *n_dev;
    for (uint32_t r = blockIdx.x * SKY_WG + threadIdx.x; r < n; r += gridDim.x * SKY_WG) {
        keys[r] = ukey[r];
        vals[r] = r;
    }
}

template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_u_regather(const uint32_t *__restrict__ urec,
                                                      const uint32_t *__restrict__ uid,
                                                      const uint32_t *__restrict__ vals, const uint32_t *n_dev,
                                                      uint32_t *__restrict__ rec, uint32_t *__restrict__ sid,
                                                      uint32_t *poff)
{
    const uint32_t n = *n_dev;
    if (blockIdx.x == 0 && threadIdx.x == 0) { poff[0] = 0; poff[1] = n; }
    for (uint32_t r = blockIdx.x * SKY_WG + threadIdx.x; r < n; r += gridDim.x * SKY_WG) {
        const uint32_t v = vals[r];
        const uint4 *s = reinterpret_cast<const uint4 *>(urec + (size_t)v * DP);
        uint4 *d = reinterpret_cast<uint4 *>(rec + (size_t)r * DP);
#pragma unroll
        for (int k = 0; k < DP / 4; ++k) d[k] = s[k];
        sid[r] = uid[v];
    }
}

hipError_t launch_u_sort_prep(const uint64_t *ukey, const uint32_t *n_dev, uint32_t n_max, uint64_t *keys,
                              uint32_t *vals, hipStream_t s)
{
    uint32_t blocks = (n_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_u_sort_prep, dim3(blocks), dim3(SKY_WG), 0, s, ukey, n_dev, keys, vals);
    return hipGetLastError();
}

hipError_t launch_u_regather(int d, const uint32_t *urec, const uint32_t *uid, const uint32_t *vals,
                             const uint32_t *n_dev, uint32_t n_max, uint32_t *rec, uint32_t *sid, uint32_t *poff,
                             hipStream_t s)
{
    uint32_t blocks = (n_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    const int DP = sky_dp(d);
#define RG_CASE(X)                                                                                          \
    case X:                                                                                                 \
        hipLaunchKernelGGL(k_u_regather<X>, dim3(blocks), dim3(SKY_WG), 0, s, urec, uid, vals, n_dev, rec, \
                           sid, poff);                                                                      \
        break;
    switch (DP) {
        RG_CASE(4) RG_CASE(8) RG_CASE(12) RG_CASE(16) RG_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef RG_CASE
    return hipGetLastError();
}
