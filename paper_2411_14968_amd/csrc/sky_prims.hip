// Data-movement primitives of the skyline path on gfx950: fills, a stable LSD
// radix sort of (uint64 key, uint32 value) pairs, stream compaction and the
// ascending id output. All sizes that depend on the data are read from device
// counters, so a launch sequence never waits for the host.
#include "sky_internal.h"

// ------------------------------------------------------------------ fill
__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Several fills in one launch: segment i sets p[i][0 .. n[i]) to v[i].
__global__ void k_fill_multi(FillSet f)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (int q = 0; q < f.cnt; ++q)
        for (size_t j = i; j < f.n[q]; j += stride) f.p[q][j] = f.v[q];
}

hipError_t launch_fill_multi(const FillSet &f, hipStream_t s)
{
    size_t most = 0;
    for (int q = 0; q < f.cnt; ++q) most = f.n[q] > most ? f.n[q] : most;
    if (most == 0) return hipSuccess;
    size_t blocks = (most + SKY_WG - 1) / SKY_WG;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_multi, dim3((unsigned)blocks), dim3(SKY_WG), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(SKY_WG), 0, s, p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ uint64_t lanemask_lt64()
{
    const uint32_t lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Exclusive scan of one uint32 per thread over a 256-thread block. Returns the
// exclusive prefix; *total receives the block sum. Uses s_tmp[4].
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *s_tmp, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wv] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t t = s_tmp[w];
        if (w < wv) base += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// ------------------------------------------------------------------ radix sort
// Pass over bits [shift, shift+8): per-workgroup digit histograms of a
// contiguous segment, a single-workgroup exclusive scan in (digit, workgroup)
// order, then a stable scatter in which each workgroup ranks its elements in
// input order (wave ballots give the rank among equal digits inside a wave)
// and writes each tile of keys digit by digit.
template <typename KT>
__global__ __launch_bounds__(SKY_WG) void k_rs_hist(const KT *__restrict__ keys,
                                                   const uint32_t *n_dev, uint32_t n_const, int shift,
                                                   uint32_t *hist, int G)
{
    __shared__ uint32_t h[256];
    const uint32_t n = n_dev ? *n_dev : n_const;
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t seg = (n + G - 1) / G;
    const uint64_t b0 = (uint64_t)blockIdx.x * seg;
    const uint64_t e0 = b0 + seg < n ? b0 + seg : n;
    for (uint64_t i = b0 + threadIdx.x; i < e0; i += SKY_WG)
        atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
}


// Exclusive scan of a short array in place (one workgroup; for per-workgroup
// counts); total (nullable) receives the sum.
__global__ __launch_bounds__(1024) void k_scan_small(uint32_t *a, uint32_t cnt, uint32_t *total)
{
    __shared__ uint32_t s[1024];
    const uint32_t per = (cnt + 1023) / 1024;
    const uint32_t b = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t i = 0; i < per && b + i < cnt; ++i) sum += a[b + i];
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (total && threadIdx.x == 1023) *total = s[1023];
    uint32_t run = s[threadIdx.x] - sum;
    for (uint32_t i = 0; i < per && b + i < cnt; ++i) {
        const uint32_t v = a[b + i];
        a[b + i] = run;
        run += v;
    }
}

// Exclusive scan of cnt counts in place, over many workgroups of 1024: each
// workgroup scans its 1024 counts (coalesced) and exchanges its total into
// bpre[] atomically; the last workgroup to finish (atomic ticket, no waiting)
// reads the totals with atomic loads, turns them into an exclusive prefix and
// resets the ticket. The scanned value of entry i
// is a[i] + bpre[i / 1024].
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *a, uint32_t cnt, uint32_t *bpre, uint32_t *ticket)
{
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_last;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t i = blockIdx.x * 1024 + t;
    const uint32_t v = i < cnt ? a[i] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) s_w[wv] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t w = 0; w < 16; ++w) {
        const uint32_t c = s_w[w];
        if (w < wv) base += c;
        tot += c;
    }
    if (i < cnt) a[i] = base + x - v;
    if (t == 0) {
        sky_consume(atomicExch(&bpre[blockIdx.x], tot));
        s_last = (atomicAdd(ticket, 1u) == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_last)) {
        const uint32_t nb = gridDim.x;   // <= 1024
        const uint32_t b = t < nb ? __hip_atomic_load(&bpre[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        uint32_t y = b;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t z = __shfl_up(y, o, 64);
            if (lane >= (uint32_t)o) y += z;
        }
        __syncthreads();
        if (lane == 63) s_w[wv] = y;
        __syncthreads();
        uint32_t bb = 0;
        for (uint32_t w = 0; w < wv; ++w) bb += s_w[w];
        if (t < nb) bpre[t] = bb + y - b;
        if (t == 0) *ticket = 0u;
    }
}

// One chunk of SKY_WG keys of a scatter pass (all threads, in input order):
// each key's rank among equal digits of its wave from 8 ballots, the wave
// counts per digit, then the stores at the digit's running offset.
template <typename KT>
__device__ __forceinline__ void rs_scatter_chunk(KT key, uint32_t val, bool valid, int shift, uint32_t *s_off,
                                                 uint32_t (*s_wc)[256], KT *__restrict__ kout,
                                                 uint32_t *__restrict__ vout)
{
    const int t = threadIdx.x, wv = t >> 6;
    const uint32_t dig = valid ? (uint32_t)(key >> shift) & 255u : 0u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (dig >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    const uint64_t lower = peers & lanemask_lt64();
    const uint32_t rank = (uint32_t)__popcll(lower);
    if (valid && lower == 0) s_wc[wv][dig] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
        uint32_t pos = s_off[dig] + rank;
        for (int w = 0; w < wv; ++w) pos += s_wc[w][dig];
        kout[pos] = key;
        vout[pos] = val;
    }
    __syncthreads();
    s_off[t] += s_wc[0][t] + s_wc[1][t] + s_wc[2][t] + s_wc[3][t];
    s_wc[0][t] = s_wc[1][t] = s_wc[2][t] = s_wc[3][t] = 0;
    __syncthreads();
}

// A workgroup scatters its segment chunk by chunk, in order (stable). The
// chunks' loads run RS_RING chunks ahead through a ring of registers, so a
// long segment does not wait for each chunk's load in turn. This form, with
// fewer barriers per key, is used for short segments (sorts of up to 4M keys).
#define RS_RING 4
template <typename KT>
__global__ __launch_bounds__(SKY_WG) void k_rs_scatter_chunks(const KT *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin,
                                                      KT *__restrict__ kout,
                                                      uint32_t *__restrict__ vout,
                                                      const uint32_t *n_dev, uint32_t n_const,
                                                      int shift, const uint32_t *__restrict__ offs,
                                                      const uint32_t *__restrict__ bpre, int G)
{
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_wc[4][256];
    const uint32_t n = n_dev ? *n_dev : n_const;
    const int t = threadIdx.x;
    const uint32_t idx = t * G + blockIdx.x;
    s_off[t] = offs[idx] + bpre[idx >> 10];
    s_wc[0][t] = s_wc[1][t] = s_wc[2][t] = s_wc[3][t] = 0;
    __syncthreads();
    const uint32_t seg = (n + G - 1) / G;
    const uint64_t b0 = (uint64_t)blockIdx.x * seg;
    const uint64_t e0 = b0 + seg < n ? b0 + seg : n;
    const uint32_t nch = e0 > b0 ? (uint32_t)((e0 - b0 + SKY_WG - 1) / SKY_WG) : 0u;   // uniform
    KT kk[RS_RING];
    uint32_t vv[RS_RING];
#pragma unroll
    for (int r = 0; r < RS_RING; ++r) {
        const uint64_t i = b0 + (uint64_t)r * SKY_WG + t;
        const bool in = i < e0;
        kk[r] = in ? kin[i] : (KT)0;
        vv[r] = in ? vin[i] : 0u;
    }
    for (uint32_t c0 = 0; c0 < nch; c0 += RS_RING) {
#pragma unroll
        for (int r = 0; r < RS_RING; ++r) {
            const uint32_t c = c0 + r;
            if (c < nch) {   // uniform
                const KT key = kk[r];
                const uint32_t val = vv[r];
                const bool valid = b0 + (uint64_t)c * SKY_WG + t < e0;
                // refill this slot with chunk c + RS_RING before the chunk is scattered
                const uint64_t inx = b0 + (uint64_t)(c + RS_RING) * SKY_WG + t;
                const bool in = inx < e0;
                kk[r] = in ? kin[inx] : (KT)0;
                vv[r] = in ? vin[inx] : 0u;
                rs_scatter_chunk<KT>(key, val, valid, shift, s_off, s_wc, kout, vout);
            }
        }
    }
}

// The same, tile by tile, for long segments (sorts of more than 4M keys). A tile of
// RS_TPT * SKY_WG keys is ranked in LDS -- each key's rank among the tile's
// equal digits in input order: ballots inside a wave, per-wave counts across
// the waves and chunks -- then reordered there by digit and written out so
// that the keys of one digit leave as one run of consecutive addresses: the
// stores of a wave cover a few runs instead of up to 64 scattered words.
#define RS_TPT 4
template <typename KT>
__global__ __launch_bounds__(SKY_WG) void k_rs_scatter(const KT *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin,
                                                      KT *__restrict__ kout,
                                                      uint32_t *__restrict__ vout,
                                                      const uint32_t *n_dev, uint32_t n_const,
                                                      int shift, const uint32_t *__restrict__ offs,
                                                      const uint32_t *__restrict__ bpre, int G)
{
    constexpr uint32_t TILE = RS_TPT * SKY_WG;
    __shared__ uint32_t s_off[256];     // global position of each digit's next key
    __shared__ uint32_t s_run[256];     // keys of each digit in the tile so far
    __shared__ uint32_t s_toff[256];    // each digit's first position in the tile
    __shared__ uint32_t s_wc[4][256];   // per-wave digit counts of the current chunk
    __shared__ uint32_t s_tmp[4];
    __shared__ KT s_k[TILE];
    __shared__ uint32_t s_v[TILE];
    const uint32_t n = n_dev ? *n_dev : n_const;
    const int t = threadIdx.x, wv = t >> 6;
    const uint32_t idx = t * G + blockIdx.x;
    s_off[t] = offs[idx] + bpre[idx >> 10];
    s_run[t] = 0;
    s_wc[0][t] = s_wc[1][t] = s_wc[2][t] = s_wc[3][t] = 0;
    __syncthreads();
    const uint32_t seg = (n + G - 1) / G;
    const uint64_t b0 = (uint64_t)blockIdx.x * seg;
    const uint64_t e0 = b0 + seg < n ? b0 + seg : n;
    for (uint64_t tb = b0; tb < e0; tb += TILE) {   // uniform
        KT k[RS_TPT];
        uint32_t v[RS_TPT], dg[RS_TPT], rk[RS_TPT];
#pragma unroll
        for (int j = 0; j < RS_TPT; ++j) {   // all loads of the tile issued together
            const uint64_t i = tb + (uint64_t)j * SKY_WG + t;
            const bool in = i < e0;
            k[j] = in ? kin[i] : (KT)0;
            v[j] = in ? vin[i] : 0u;
            dg[j] = in ? (uint32_t)(k[j] >> shift) & 255u : 256u;
        }
#pragma unroll
        for (int j = 0; j < RS_TPT; ++j) {   // chunk j: ranks after every earlier key of the tile
            const bool valid = dg[j] < 256u;
            const uint32_t d = valid ? dg[j] : 0u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint64_t lower = peers & lanemask_lt64();
            if (valid && lower == 0) s_wc[wv][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            rk[j] = 0;
            if (valid) {
                uint32_t r = s_run[d] + (uint32_t)__popcll(lower);
                for (int w = 0; w < wv; ++w) r += s_wc[w][d];
                rk[j] = r;
            }
            __syncthreads();
            s_run[t] += s_wc[0][t] + s_wc[1][t] + s_wc[2][t] + s_wc[3][t];
            s_wc[0][t] = s_wc[1][t] = s_wc[2][t] = s_wc[3][t] = 0;
            __syncthreads();
        }
        uint32_t tot;
        s_toff[t] = block_excl_scan256(s_run[t], s_tmp, &tot);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RS_TPT; ++j)   // the tile in digit order
            if (dg[j] < 256u) {
                const uint32_t p = s_toff[dg[j]] + rk[j];
                s_k[p] = k[j];
                s_v[p] = v[j];
            }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RS_TPT; ++j) {   // tile position m of digit d goes to s_off[d] + (m - s_toff[d])
            const uint32_t m = (uint32_t)j * SKY_WG + t;
            if (m < tot) {
                const KT key = s_k[m];
                const uint32_t d = (uint32_t)(key >> shift) & 255u;
                const uint32_t g = s_off[d] + (m - s_toff[d]);
                kout[g] = key;
                vout[g] = s_v[m];
            }
        }
        __syncthreads();
        s_off[t] += s_run[t];
        s_run[t] = 0;
        __syncthreads();
    }
}

template <typename KT>
static hipError_t radix_sort_t(SortBufs &b, const uint32_t *n_dev, uint32_t n_max, int bit_lo, int bit_hi,
                               hipStream_t s)
{
    if (n_max == 0) return hipSuccess;
    const int passes = (bit_hi - bit_lo + 7) / 8;
    const int G = b.G;
    // from 4M keys on, the workgroup count stops growing (1024), so segments are long: tiles
    const bool tiles = n_max >= (4u << 20);
    KT *ki = reinterpret_cast<KT *>(b.kA), *ko = reinterpret_cast<KT *>(b.kB);
    uint32_t *vi = b.vA, *vo = b.vB;
    for (int p = 0; p < passes; ++p) {
        const int shift = bit_lo + 8 * p;
        hipLaunchKernelGGL(k_rs_hist<KT>, dim3(G), dim3(SKY_WG), 0, s, ki, n_dev, n_max, shift, b.hist, G);
        hipLaunchKernelGGL(k_scan_blocks, dim3((256 * G + 1023) / 1024), dim3(1024), 0, s, b.hist,
                           (uint32_t)(256 * G), b.bpre, b.ticket);
        if (tiles)
            hipLaunchKernelGGL(k_rs_scatter<KT>, dim3(G), dim3(SKY_WG), 0, s, ki, vi, ko, vo, n_dev, n_max, shift,
                               b.hist, b.bpre, G);
        else
            hipLaunchKernelGGL(k_rs_scatter_chunks<KT>, dim3(G), dim3(SKY_WG), 0, s, ki, vi, ko, vo, n_dev, n_max,
                               shift, b.hist, b.bpre, G);
        KT *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
    }
    if (passes & 1) {   // the result is in the second pair: swap the roles so that kA / vA name it
        b.kB = b.kA; b.kA = reinterpret_cast<uint64_t *>(ki);
        b.vB = b.vA; b.vA = vi;
    }
    return hipGetLastError();
}

hipError_t launch_radix_sort(SortBufs &b, const uint32_t *n_dev, uint32_t n_max, int bit_lo, int bit_hi,
                             hipStream_t s)
{
    return radix_sort_t<uint64_t>(b, n_dev, n_max, bit_lo, bit_hi, s);
}

// The same sort over 32-bit keys held in the same buffers (bit_hi <= 32): half
// the key bytes of every pass.
hipError_t launch_radix_sort32(SortBufs &b, const uint32_t *n_dev, uint32_t n_max, int bit_lo, int bit_hi,
                               hipStream_t s)
{
    if (bit_hi > 32) return hipErrorInvalidValue;
    return radix_sort_t<uint32_t>(b, n_dev, n_max, bit_lo, bit_hi, s);
}
int sort_groups(uint32_t n_max)
{
    uint32_t g = (n_max + 4095) / 4096;
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    return (int)g;
}

// ------------------------------------------------------------------ output
// Skyline bitmap over original ids -> ascending int64 ids. Each workgroup owns
// 1024 consecutive bitmap words (4 per thread).
#define OUT_WORDS_PER_WG 1024

__global__ __launch_bounds__(SKY_WG) void k_out_count(const uint32_t *__restrict__ bits, uint32_t nwords,
                                                     uint32_t *wg_cnt)
{
    __shared__ uint32_t s_tmp[4];
    const uint32_t w0 = blockIdx.x * OUT_WORDS_PER_WG + threadIdx.x * 4;
    uint32_t c = 0;
    for (int q = 0; q < 4; ++q)
        if (w0 + q < nwords) c += __popc(bits[w0 + q]);
    uint32_t tot;
    block_excl_scan256(c, s_tmp, &tot);
    if (threadIdx.x == 0) wg_cnt[blockIdx.x] = tot;
}

// wg_cnt: the per-workgroup counts, or (scanned) their exclusive prefix. With
// counts, each workgroup sums those before its own (up to a few thousand), so
// no scan launch sits between the two kernels.
__global__ __launch_bounds__(SKY_WG) void k_out_write(const uint32_t *__restrict__ bits, uint32_t nwords,
                                                     const uint32_t *__restrict__ wg_cnt, int scanned, uint32_t nwg,
                                                     int64_t *ids, uint32_t cap, uint32_t *ctrl)
{
    __shared__ uint32_t s_tmp[4];
    uint32_t off;
    if (scanned) {
        off = wg_cnt[blockIdx.x];
    } else {
        uint32_t before = 0;
        for (uint32_t j = threadIdx.x; j < blockIdx.x; j += SKY_WG) before += wg_cnt[j];
        block_excl_scan256(before, s_tmp, &off);
    }
    const uint32_t w0 = blockIdx.x * OUT_WORDS_PER_WG + threadIdx.x * 4;
    uint32_t wv[4], c = 0;
    for (int q = 0; q < 4; ++q) {
        wv[q] = (w0 + q < nwords) ? bits[w0 + q] : 0u;
        c += __popc(wv[q]);
    }
    uint32_t tot;
    uint32_t pos = off + block_excl_scan256(c, s_tmp, &tot);
    for (int q = 0; q < 4; ++q) {
        uint32_t w = wv[q];
        while (w) {
            const int b = __ffs(w) - 1;
            if (pos < cap) ids[pos] = (int64_t)(w0 + q) * 32 + b;
            ++pos;
            w &= w - 1;
        }
    }
    if (blockIdx.x == nwg - 1 && threadIdx.x == 0) ctrl[C_NSKY] = off + tot;
}

// ids: device-accessible destination (device memory or mapped pinned host
// memory) with room for cap ids; ids past cap are counted but not written.
hipError_t launch_output(const uint32_t *skybits, uint32_t n, uint32_t *wg_cnt, int64_t *ids, uint32_t cap,
                         uint32_t *ctrl, hipStream_t s)
{
    const uint32_t nwords = (n + 31) / 32;
    if (nwords == 0) return hipSuccess;
    const uint32_t nwg = (nwords + OUT_WORDS_PER_WG - 1) / OUT_WORDS_PER_WG;
    hipLaunchKernelGGL(k_out_count, dim3(nwg), dim3(SKY_WG), 0, s, skybits, nwords, wg_cnt);
    // up to 4096 workgroups (134M points) each sums the counts before its own; beyond, one scan launch
    const int scanned = nwg > 4096 ? 1 : 0;
    if (scanned) hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, wg_cnt, nwg, (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_out_write, dim3(nwg), dim3(SKY_WG), 0, s, skybits, nwords, wg_cnt, scanned, nwg, ids, cap,
                       ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------------------ compaction + presort keys
// Survivors of the filters get the presort key
//   (partition id : pbits | Q : kbits - pbits), kbits 24, 32 or 64,
// Q either the top bits of map(score) or the Z-order code of the quantised
// coordinates (zq given). Both Q are monotone, so s dominating t gives
// Q(s) <= Q(t): sorted by the key, every dominator of a point comes before it
// or has the same key (the dominance kernels also test the equal-key run). The
// Z order keeps nearby points together, which makes the lower corners of
// record blocks tight for the dominance scans.
// Emission keeps input order (stable), so equal keys stay in id order.

// Survivors per emission segment: G segments of seg = ceil(n / G) points, one
// workgroup each. The emission kernel sums the counts before its own segment.
__global__ __launch_bounds__(SKY_WG) void k_count_alive(const uint8_t *__restrict__ alive, uint32_t n,
                                                       uint32_t *wg_cnt, int G)
{
    __shared__ uint32_t s_tmp[4];
    const uint32_t seg = (n + G - 1) / G;
    const uint64_t b0 = (uint64_t)blockIdx.x * seg;
    const uint64_t e0 = b0 + seg < n ? b0 + seg : n;
    uint32_t c = 0;
    for (uint64_t i = b0 + threadIdx.x; i < e0; i += SKY_WG) c += alive[i] ? 1u : 0u;
    uint32_t tot;
    block_excl_scan256(c, s_tmp, &tot);
    if (threadIdx.x == 0) wg_cnt[blockIdx.x] = tot;
}

template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_emit_keys(const float *__restrict__ score,
                                                     const float *__restrict__ zq, int zb, int nz,
                                                     const float *__restrict__ pts, uint32_t n, int d,
                                                     const uint8_t *__restrict__ alive,
                                                     const uint32_t *__restrict__ part, int pbits,
                                                     int qbits, int kbits, int tie, int k32, const uint32_t *__restrict__ wg_cnt,
                                                     int G, uint64_t *keys, uint32_t *vals, uint32_t *ctrl,
                                                     uint32_t *__restrict__ rec_stage, uint32_t *__restrict__ id_stage)
{
    constexpr int ND = DP - 2;
    __shared__ uint32_t s_tmp[4];
    const uint32_t seg = (n + G - 1) / G;
    const uint64_t b0 = (uint64_t)blockIdx.x * seg;
    const uint64_t e0 = b0 + seg < n ? b0 + seg : n;
    // this segment's first output position: the survivors of the segments before it (G <= 1024)
    uint32_t before = 0;
    for (uint32_t j = threadIdx.x; j < blockIdx.x; j += SKY_WG) before += wg_cnt[j];
    uint32_t pos;
    block_excl_scan256(before, s_tmp, &pos);
    for (uint64_t base = b0; base < e0; base += SKY_WG) {
        const uint64_t i = base + threadIdx.x;
        const bool a = (i < e0) && alive[i];
        uint32_t tot;
        const uint32_t r = block_excl_scan256(a ? 1u : 0u, s_tmp, &tot);
        if (a) {
            // all coordinate loads issued together (compile-time count, clamped index)
            float x[ND];
#pragma unroll
            for (int k = 0; k < ND; ++k) x[k] = pts[(size_t)(k < d ? k : d - 1) * n + i];
            uint64_t q;
            if (zq) {
                const float qmax = (float)((1u << zb) - 1u);
                uint64_t z = 0;
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    if (k >= nz) continue;
                    float t = (x[k] - zq[k]) * zq[16 + k];
                    t = fminf(fmaxf(t, 0.0f), qmax);   // fmaxf maps NaN to 0
                    const uint32_t qk = (uint32_t)t;
                    for (int l = 0; l < zb; ++l) z |= (uint64_t)((qk >> l) & 1u) << (l * nz + (nz - 1 - k));
                }
                q = z;
            } else {
                q = (uint64_t)(ordmap(score[i]) >> (32 - qbits));
            }
            uint64_t key = q;
            if (pbits) key |= (uint64_t)part[i] << (kbits - pbits);
            // tie word: below the Z-order code, the score (float32 sum, monotone
            // too), so that points in one Z-order cell are ordered by it and runs
            // of equal keys stay short; the key is then kbits + 32 bits wide
            if (tie) key = (key << 32) | ordmap(score[i]);
            if (k32)   // the whole key fits 32 bits: stored as one word (the sort then moves half the bytes)
                reinterpret_cast<uint32_t *>(keys)[pos + r] = (uint32_t)key;
            else
                keys[pos + r] = key;
            if (rec_stage) {
                // the survivor's record and id at its compacted position; the sort
                // carries that position, and the gather reads one record per output
                uint32_t w[DP];
                uint64_t K = 0;
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    w[k] = (k < d) ? ordmap(x[k]) : 0u;
                    K += w[k];
                }
                w[DP - 2] = (uint32_t)K;
                w[DP - 1] = (uint32_t)(K >> 32);
                uint4 *dst = reinterpret_cast<uint4 *>(rec_stage + (size_t)(pos + r) * DP);
#pragma unroll
                for (int k = 0; k < DP / 4; ++k)
                    dst[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
                id_stage[pos + r] = (uint32_t)i;
                vals[pos + r] = pos + r;
            } else {
                vals[pos + r] = (uint32_t)i;
            }
        }
        pos += tot;
    }
    if (blockIdx.x == G - 1 && threadIdx.x == 0) ctrl[C_NSURV] = pos;
}

hipError_t launch_emit_keys(const float *score, const float *zq, const float *pts, uint32_t n, int d,
                            const uint8_t *alive, const uint32_t *part, int pbits, uint32_t *wg_cnt,
                            uint64_t *keys, uint32_t *vals, uint32_t *ctrl, hipStream_t s, uint32_t *rec_stage,
                            uint32_t *id_stage, int kbits, int tie, int k32)
{
    if (n == 0) return hipSuccess;
    const int qbits = kbits - pbits;
    if (qbits < 1) return hipErrorInvalidValue;
    int zb = 0, nz = 0;
    if (zq) zorder_layout(d, qbits, &zb, &nz);
    int G = (int)((n + 1023) / 1024);   // segments of at least 1024 points, at most 1024 of them
    if (G > 1024) G = 1024;
    hipLaunchKernelGGL(k_count_alive, dim3(G), dim3(SKY_WG), 0, s, alive, n, wg_cnt, G);
    const int DP = sky_dp(d);
#define E_CASE(X)                                                                                                  \
    case X:                                                                                                        \
        hipLaunchKernelGGL(k_emit_keys<X>, dim3(G), dim3(SKY_WG), 0, s, score, zq, zb, nz, pts, n, d, alive, part, \
                           pbits, qbits, kbits, tie, k32, wg_cnt, G, keys, vals, ctrl, rec_stage, id_stage);       \
        break;
    switch (DP) {
        E_CASE(4) E_CASE(8) E_CASE(12) E_CASE(16) E_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef E_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------ gather
// Sorted order -> AoS records, original ids, Q keys without the partition
// bits, and partition offsets poff[0..np] (survivors of partition j occupy
// [poff[j], poff[j+1])).
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_gather(const float *__restrict__ pts, uint32_t n, int d,
                                                  const uint64_t *__restrict__ keys,
                                                  const uint32_t *__restrict__ vals, const uint32_t *n_dev,
                                                  int pbits, int np, uint32_t *__restrict__ rec,
                                                  uint32_t *__restrict__ sid, uint64_t *__restrict__ skey,
                                                  uint32_t *__restrict__ poff, const uint32_t *__restrict__ rec_stage,
                                                  const uint32_t *__restrict__ id_stage, int kbits, int k32)
{
    const uint32_t ns = *n_dev;
    const uint32_t *keys32 = reinterpret_cast<const uint32_t *>(keys);
    const uint64_t pmask = kbits - pbits >= 64 ? ~0ull : (1ull << (kbits - pbits)) - 1;
    if (ns == 0) {
        if (blockIdx.x == 0)
            for (int j = threadIdx.x; j <= np; j += SKY_WG) poff[j] = 0;
        return;
    }
    for (uint32_t r = blockIdx.x * SKY_WG + threadIdx.x; r < ns; r += gridDim.x * SKY_WG) {
        const uint32_t v = vals[r];
        const uint64_t key = k32 ? (uint64_t)keys32[r] : keys[r];
        uint32_t w[DP];
        uint32_t id;
        if (rec_stage) {   // v: compacted position of a record staged by the key emission
            const uint4 *src = reinterpret_cast<const uint4 *>(rec_stage + (size_t)v * DP);
#pragma unroll
            for (int k = 0; k < DP / 4; ++k) {
                const uint4 q4 = src[k];
                w[4 * k] = q4.x; w[4 * k + 1] = q4.y; w[4 * k + 2] = q4.z; w[4 * k + 3] = q4.w;
            }
            id = id_stage[v];
        } else {           // v: input id
            id = v;
            uint64_t K = 0;
            float x[DP - 2];
#pragma unroll
            for (int k = 0; k < DP - 2; ++k) x[k] = pts[(size_t)(k < d ? k : d - 1) * n + id];
#pragma unroll
            for (int k = 0; k < DP - 2; ++k) {
                w[k] = (k < d) ? ordmap(x[k]) : 0u;
                K += w[k];
            }
            w[DP - 2] = (uint32_t)K;
            w[DP - 1] = (uint32_t)(K >> 32);
        }
        uint4 *dst = reinterpret_cast<uint4 *>(rec + (size_t)r * DP);
#pragma unroll
        for (int k = 0; k < DP / 4; ++k) dst[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
        sid[r] = id;
        skey[r] = key & pmask;
        const uint32_t pj = pbits ? (uint32_t)(key >> (kbits - pbits)) : 0u;
        const uint32_t pprev = (r == 0) ? 0xffffffffu
                                        : (pbits ? (uint32_t)((k32 ? (uint64_t)keys32[r - 1] : keys[r - 1]) >>
                                                              (kbits - pbits))
                                                 : 0u);
        if (r == 0) {
            for (uint32_t j = 0; j <= pj; ++j) poff[j] = 0;
        } else if (pprev != pj) {
            for (uint32_t j = pprev + 1; j <= pj; ++j) poff[j] = r;
        }
        if (r == ns - 1)
            for (uint32_t j = pj + 1; j <= (uint32_t)np; ++j) poff[j] = ns;
    }
}

hipError_t launch_gather(const float *pts, uint32_t n, int d, const uint64_t *keys, const uint32_t *vals,
                         const uint32_t *n_dev, uint32_t n_max, int pbits, int np, uint32_t *rec,
                         uint32_t *sid, uint64_t *skey, uint32_t *poff, hipStream_t s, const uint32_t *rec_stage,
                         const uint32_t *id_stage, int kbits, int k32)
{
    uint32_t blocks = (n_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    const int DP = sky_dp(d);
#define G_CASE(X)                                                                                              \
    case X:                                                                                                    \
        hipLaunchKernelGGL(k_gather<X>, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, d, keys, vals, n_dev, pbits, \
                           np, rec, sid, skey, poff, rec_stage, id_stage, kbits, k32);                         \
        break;
    switch (DP) {
        G_CASE(4) G_CASE(8) G_CASE(12) G_CASE(16) G_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef G_CASE
    return hipGetLastError();
}

hipError_t launch_scan_counts(uint32_t *a, uint32_t n, uint32_t *tmp2, uint32_t *total, hipStream_t s)
{
    (void)tmp2;
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, a, n, total);
    return hipGetLastError();
}
