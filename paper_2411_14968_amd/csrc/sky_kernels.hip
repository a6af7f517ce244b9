// Skyline kernels for gfx950: ingest and validation, Grid Filtering,
// representative selection and filtering, partition assignment, the local
// skyline (SFS semantics) and the NoSeq merge.
//
// Dominance (Def. 1) is evaluated on order-preserving uint32 images of the
// coordinates, so every test is an exact integer comparison.
#include "sky_internal.h"
#include "sky_domtest.h"

__device__ __forceinline__ uint64_t lmask_lt()
{
    const uint32_t lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Grid cell of coordinate x with m slices: min(floor(x m), m - 1), exact in
// float64 (a float32 times a small integer is exact). Values outside [0,1]
// (already flagged as an error) are clamped so every index stays in bounds.
__device__ __forceinline__ uint32_t grid_digit(float x, int m)
{
    const double v = (double)x * (double)m;
    int c = (v >= 0.0) ? (int)floor(v) : 0;
    if (c > m - 1) c = m - 1;
    if (c < 0) c = 0;
    return (uint32_t)c;
}

// ------------------------------------------------------------------ ingest
// Validates coordinates, writes the float32 sequential coordinate sum (the
// Sorted-representative and presort score) and marks Grid-Filtering cells.
// Each thread takes INGEST_PPT points per pass, so the per-workgroup bounds
// reduction is paid once per INGEST_PPT * SKY_WG points.
#define INGEST_PPT 4
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_ingest(const float *__restrict__ pts, uint32_t n, int d,
                                                  int need_range, float *__restrict__ score, int gf_on,
                                                  GridSpec gg, uint32_t *occ, uint32_t *ctrl, float *bnd)
{
    constexpr int ND = DP - 2;
    uint32_t err = 0;
    float lo[ND], hi[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        lo[k] = __builtin_huge_valf();
        hi[k] = -__builtin_huge_valf();
    }
    for (uint32_t b0 = blockIdx.x * SKY_WG * INGEST_PPT; b0 < n; b0 += gridDim.x * SKY_WG * INGEST_PPT) {
      // the coordinate loads of all INGEST_PPT points issued together (compile-time
      // count, clamped index); then the points one by one
      float xs[INGEST_PPT][ND];
#pragma unroll
      for (int q = 0; q < INGEST_PPT; ++q) {
          const uint32_t i = b0 + q * SKY_WG + threadIdx.x, ic = i < n ? i : n - 1;
#pragma unroll
          for (int k = 0; k < ND; ++k) xs[q][k] = pts[(size_t)(k < d ? k : d - 1) * n + ic];
      }
#pragma unroll
      for (int q = 0; q < INGEST_PPT; ++q) {
        const uint32_t i = b0 + q * SKY_WG + threadIdx.x;
        if (i >= n) break;
        const float(&x)[ND] = xs[q];
        float s = 0.0f;
        uint32_t cell = 0, mult = 1;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            if (k >= d) continue;
            const uint32_t u = __float_as_uint(x[k]);
            if ((u & 0x7f800000u) == 0x7f800000u) err |= 1u;
            else if (need_range && !(x[k] >= 0.0f && x[k] <= 1.0f)) err |= 2u;
            s = (k == 0) ? x[k] : s + x[k];
            lo[k] = fminf(lo[k], x[k]);
            hi[k] = fmaxf(hi[k], x[k]);
            if (gf_on) {
                cell += grid_digit(x[k], gg.m[k]) * mult;
                mult *= (uint32_t)gg.m[k];
            }
        }
        if (score) score[i] = s;
        if (gf_on) {
            const uint32_t bit = 1u << (cell & 31);
            if (!(occ[cell >> 5] & bit)) atomicOr(&occ[cell >> 5], bit);
        }
      }
    }
    if (err) atomicOr(&ctrl[C_ERR], err);
    if (bnd) {
        // per-workgroup bounds of every coordinate: bnd[wg*32 + k] = min, [.. + 16 + k] = max
        __shared__ float s_b[4][32];
        const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            float l = lo[k], h = hi[k];
            for (int o = 32; o > 0; o >>= 1) {
                l = fminf(l, __shfl_xor(l, o, 64));
                h = fmaxf(h, __shfl_xor(h, o, 64));
            }
            if (lane == 0) { s_b[wv][k] = l; s_b[wv][16 + k] = h; }
        }
        __syncthreads();
        if (threadIdx.x < (uint32_t)d) {
            const int k = threadIdx.x;
            bnd[blockIdx.x * 32 + k] = fminf(fminf(s_b[0][k], s_b[1][k]), fminf(s_b[2][k], s_b[3][k]));
            bnd[blockIdx.x * 32 + 16 + k] =
                fmaxf(fmaxf(s_b[0][16 + k], s_b[1][16 + k]), fmaxf(s_b[2][16 + k], s_b[3][16 + k]));
        }
    }
}

static uint32_t ingest_blocks(uint32_t n)
{
    uint32_t blocks = (n + SKY_WG * INGEST_PPT - 1) / (SKY_WG * INGEST_PPT);
    return blocks > SKY_INGEST_MAX_WG ? SKY_INGEST_MAX_WG : blocks;
}

hipError_t launch_ingest(const float *pts, uint32_t n, int d, int need_range, float *score, int gf_on,
                         const GridSpec &gg, uint32_t *occ, uint32_t *ctrl, float *bnd, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int DP = sky_dp(d);
#define I_CASE(X)                                                                                            \
    case X:                                                                                                  \
        hipLaunchKernelGGL(k_ingest<X>, dim3(ingest_blocks(n)), dim3(SKY_WG), 0, s, pts, n, d, need_range,   \
                           score, gf_on, gg, occ, ctrl, bnd);                                                \
        break;
    switch (DP) {
        I_CASE(4) I_CASE(8) I_CASE(12) I_CASE(16) I_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef I_CASE
    return hipGetLastError();
}

// Z-order presort key: coordinate k is quantised to b bits as
// q_k = clamp(floor((x_k - lo_k) * scale_k), 0, 2^b - 1), scale_k = 2^b / (hi_k - lo_k)
// (0 for a constant coordinate), and the q_k of the first nz coordinates are
// bit-interleaved, most significant level first. Every step is monotone
// non-decreasing in x_k (rounded subtraction and multiplication by a
// non-negative number, floor and clamp all are), so the code never decreases
// when a coordinate grows: a monotone score in the sense of Section 2.
void zorder_layout(int d, int zbits, int *b, int *nz)
{
    int bb = zbits / d;
    if (bb < 1) bb = 1;
    if (bb > 10) bb = 10;
    int z = zbits / bb;
    *b = bb;
    *nz = z < d ? z : d;
}

// One workgroup per quantised coordinate: reduce the per-workgroup bounds.
__global__ __launch_bounds__(SKY_WG) void k_zorder_scale(const float *__restrict__ bnd, uint32_t nblk, int b,
                                                        float *zq)
{
    __shared__ float s_lo[4], s_hi[4];
    const uint32_t k = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
    for (uint32_t i = threadIdx.x; i < nblk; i += SKY_WG) {
        lo = fminf(lo, bnd[i * 32 + k]);
        hi = fmaxf(hi, bnd[i * 32 + 16 + k]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) { s_lo[wv] = lo; s_hi[wv] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        lo = fminf(fminf(s_lo[0], s_lo[1]), fminf(s_lo[2], s_lo[3]));
        hi = fmaxf(fmaxf(s_hi[0], s_hi[1]), fmaxf(s_hi[2], s_hi[3]));
        const float r = hi - lo;
        float sc = (r > 0.0f && r < __builtin_huge_valf()) ? (float)(1u << b) / r : 0.0f;
        if (!(sc < __builtin_huge_valf())) sc = 0.0f;
        zq[k] = lo;
        zq[16 + k] = sc;
    }
}

hipError_t launch_zorder_scale(const float *bnd, uint32_t n, int d, int zbits, float *zq, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int b, nz;
    zorder_layout(d, zbits > 64 ? 64 : zbits, &b, &nz);
    hipLaunchKernelGGL(k_zorder_scale, dim3(nz), dim3(SKY_WG), 0, s, bnd, ingest_blocks(n), b, zq);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Grid Filtering
// Cell c is discarded when a non-empty cell is below it in every dimension
// (grid dominance, Section 3.2). P = inclusive prefix-OR of occupancy along
// every dimension; c is dominated iff all its digits are >= 1 and
// P[c - (1, ..., 1)] is set. One workgroup, occupancy held in LDS.
__global__ __launch_bounds__(1024) void k_grid_dom(const uint32_t *__restrict__ occ, uint32_t *gdom,
                                                   GridSpec g)
{
    __shared__ uint8_t P[SKY_MAX_GRID_CELLS];
    uint32_t nc = 1;
    for (int k = 0; k < g.d; ++k) nc *= (uint32_t)g.m[k];
    for (uint32_t c = threadIdx.x; c < nc; c += 1024) P[c] = (occ[c >> 5] >> (c & 31)) & 1u;
    __syncthreads();
    uint32_t stride = 1;
    for (int k = 0; k < g.d; ++k) {
        const uint32_t mk = (uint32_t)g.m[k];
        const uint32_t nlines = nc / mk;
        for (uint32_t L = threadIdx.x; L < nlines; L += 1024) {
            const uint32_t low = L % stride, high = L / stride;
            const uint32_t base = high * stride * mk + low;
            uint8_t acc = 0;
            for (uint32_t c = 0; c < mk; ++c) {
                acc |= P[base + c * stride];
                P[base + c * stride] = acc;
            }
        }
        __syncthreads();
        stride *= mk;
    }
    uint32_t diag = 0, st = 1;
    for (int k = 0; k < g.d; ++k) { diag += st; st *= (uint32_t)g.m[k]; }
    const uint32_t nw = (nc + 31) / 32;
    for (uint32_t w = threadIdx.x; w < nw; w += 1024) {
        uint32_t bits = 0;
        for (uint32_t b = 0; b < 32; ++b) {
            const uint32_t c = w * 32 + b;
            if (c >= nc) break;
            uint32_t rem = c;
            bool pos = true;
            for (int k = 0; k < g.d; ++k) {
                if (rem % (uint32_t)g.m[k] == 0) { pos = false; break; }
                rem /= (uint32_t)g.m[k];
            }
            if (pos && P[c - diag]) bits |= 1u << b;
        }
        gdom[w] = bits;
    }
}

hipError_t launch_grid_dom(const uint32_t *occ, uint32_t *gdom, const GridSpec &gg, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_dom, dim3(1), dim3(1024), 0, s, occ, gdom, gg);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Sliced boundaries by selection
// Slice j >= 1 starts at rank r_j = ceil(j N / p) of the order by x_s (Section
// 3.4). A threshold T_j with "map(x_s) >= T_j exactly when the rank is >= r_j"
// is found by a radix selection of all p - 1 ranks at once: passes over the
// 8-bit digits of the 32-bit key, each a histogram of the keys that share a
// selection's prefix so far, then a walk of that histogram to the digit whose
// bucket holds the rank. With lt_j = #{keys below the bucket}, a bucket that
// starts exactly at r_j (lt_j = r_j) settles the selection with T_j = its
// smallest possible key. After the last digit the bucket is one key value b_j;
// lt_j < r_j then means a run of equal x_s straddles the boundary (C_TIE: the
// host orders those points lexicographically instead), and otherwise T_j = b_j.
// Then slice(x) = #{j : map(x_s) >= T_j}.
//
// Every pass first rebuilds, in each workgroup, the state left by the previous
// pass's digit: from the state before it and that pass's histogram (the walk
// to the digit whose bucket holds r_j). Workgroup 0 stores the result for the
// pass after next and writes the thresholds that digit settles; a fifth step
// (one workgroup) applies the last digit and reports C_TIE. No pass waits for
// the end of another inside one launch: no ticket, no last-workgroup tail.
//
// State (uint32 words): two sets at QS_SET(s) = 256 s, each [0, 64) prefix,
// [64, 128) lt, [128, 192) each selection's histogram row in the pass that
// follows the set's writer (QS_NONE: empty slice, QS_DONE: settled), [192]
// the number of rows; then QS_HIST: three buffers of 64 rows of 256 digit
// counts, each row in SKY_HCOPY copies (row r's copy c at (r * SKY_HCOPY + c)
// * 256; workgroup b counts into copy b % SKY_HCOPY, readers sum them). Pass t counts into buffer t % 3 and clears buffer (t + 1) % 3, which
// held pass t - 2's counts; the set written during pass t is read by pass t + 1
// only. Only row 0 of buffer 0 must be zero when a selection starts (the call's
// resets): pass 0's single row.
#define QS_SET(s) ((uint32_t)(s) * 256u)
#define QS_PRE 0
#define QS_LT 64
#define QS_SO 128
#define QS_NS 192
#define QS_HIST 512
#define QS_BUF(b) (QS_HIST + (uint32_t)(b) * 64u * SKY_HCOPY * 256u)
#define QS_NONE 0xFFFFFFFFu
#define QS_DONE 0xFFFFFFFEu
static_assert(QS_HIST == SKY_QSEL_ZERO && QS_BUF(3) == SKY_QSEL_WORDS, "workspace layout");

// Pass `pass` (0..3) over the keys, or the last digit's step (pass 4, run by one
// workgroup). Each thread counts QS_KPT keys whose loads are issued first, so
// they overlap the state's. All threads of the workgroup call it; h is
// (p - 1) * 256 words of LDS. Passes run in launches of their own, or inside
// the representatives' select launches (same grid).
#define QS_KPT 16
__device__ __forceinline__ void qsel_pass_dev(const float *__restrict__ xs, uint32_t n, int p, int pass, uint32_t *qs,
                                              uint32_t *bnd, uint32_t *ctrl, uint32_t *h)
{
    __shared__ uint32_t s_pre[64], s_lt[64], s_so[64], s_slotp[64], s_ns;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t P1 = (uint32_t)p - 1;
    const bool wg0 = blockIdx.x == 0;
    const uint32_t base = blockIdx.x * SKY_WG * QS_KPT + t;
    uint32_t key[QS_KPT];
    if (pass < 4) {
#pragma unroll
        for (int k = 0; k < QS_KPT; ++k) {
            const uint32_t i = base + k * SKY_WG;
            key[k] = i < n ? ordmap(xs[i]) : 0u;
        }
    }
    // the state before the previous pass's digit; at the start (passes 0 and 1)
    // every selection with a non-empty slice is open, in row 0
    if (t < 64) {
        const bool in = t < P1;
        const uint32_t r = in ? (uint32_t)(((uint64_t)(t + 1) * n + P1) / (uint32_t)p) : 0u;   // selection j serves slice j + 1
        if (pass <= 1) {
            s_pre[t] = 0;
            s_lt[t] = 0;
            s_so[t] = in && r < n ? 0u : QS_NONE;
        } else {
            const uint32_t *st = qs + QS_SET((pass - 2) & 1);
            s_pre[t] = st[QS_PRE + t];
            s_lt[t] = st[QS_LT + t];
            s_so[t] = in ? st[QS_SO + t] : QS_NONE;
        }
        if (pass == 0 && wg0 && in) bnd[t] = 0xFFFFFFFFu;   // above every finite key: an empty slice
    }
    const uint32_t nprev = pass <= 1 ? 1u : __builtin_amdgcn_readfirstlane(qs[QS_SET((pass - 2) & 1) + QS_NS]);
    __syncthreads();
    if (pass >= 1) {
        // the previous pass's digit: its histogram rows, all loaded in one round
        const uint32_t *hp = qs + QS_BUF((pass - 1) % 3);
        for (uint32_t b = t; b < nprev * 256; b += SKY_WG) {
            const uint32_t *hr = hp + (size_t)(b >> 8) * SKY_HCOPY * 256 + (b & 255u);
            uint32_t v = 0;
#pragma unroll
            for (int c = 0; c < SKY_HCOPY; ++c) v += hr[c * 256];
            h[b] = v;
        }
        __syncthreads();
        const int shift = 24 - 8 * (pass - 1);
        // one wave per selection: each lane sums 4 bins, a wave scan finds the
        // lane whose range crosses the rank, that lane finds the bin
        for (uint32_t j = wv; j < P1; j += SKY_WG / 64) {
            const uint32_t so = s_so[j];   // wave-uniform
            if (so >= nprev) continue;
            const uint32_t *row = h + so * 256 + lane * 4;
            uint32_t c[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) c[q] = row[q];
            const uint32_t sum = c[0] + c[1] + c[2] + c[3];
            uint32_t x = sum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, 64);
                if (lane >= (uint32_t)o) x += y;
            }
            const uint32_t r = (uint32_t)(((uint64_t)(j + 1) * n + P1) / (uint32_t)p), lt0 = s_lt[j];
            const uint32_t need = r - lt0;   // keys of the prefix ranked before r_j
            const uint64_t over = __ballot(x > need);
            const uint32_t L = over ? (uint32_t)__builtin_ctzll(over) : 63u;
            if (lane == L) {
                uint32_t cum = x - sum, q = 0;
                while (q < 3 && cum + c[q] <= need) { cum += c[q]; ++q; }
                const uint32_t lt = lt0 + cum;
                const uint32_t pre = s_pre[j] | ((lane * 4 + q) << shift);
                s_pre[j] = pre;
                s_lt[j] = lt;
                if (lt == r) {   // the bucket starts at r_j: every key >= its smallest key is ranked >= r_j
                    if (wg0) bnd[j] = pre;
                    s_so[j] = QS_DONE;
                } else if (pass == 4) {   // one key value whose run straddles the boundary
                    if (wg0) atomicOr(&ctrl[C_TIE], 1u);
                    s_so[j] = QS_DONE;
                }
            }
        }
        __syncthreads();
    }
    if (pass == 4) return;
    const int shift = 24 - 8 * pass;
    // this pass's rows: the distinct prefixes of the open selections (they ascend with j)
    if (t == 0) {
        uint32_t cnt = 0, last = 0;
        for (uint32_t q = 0; q < P1; ++q) {
            if (s_so[q] >= QS_DONE) continue;
            const uint32_t v = pass == 0 ? 0u : s_pre[q] >> (shift + 8);
            if (cnt == 0 || v != last) {
                s_slotp[cnt] = v;
                last = v;
                ++cnt;
            }
            s_so[q] = cnt - 1;
        }
        s_ns = cnt;
    }
    __syncthreads();
    const uint32_t ns = __builtin_amdgcn_readfirstlane(s_ns);
    if (pass >= 1 && wg0 && t < 64) {   // for the pass after next
        uint32_t *st = qs + QS_SET((pass - 1) & 1);
        st[QS_PRE + t] = s_pre[t];
        st[QS_LT + t] = s_lt[t];
        st[QS_SO + t] = s_so[t];
        if (t == 0) st[QS_NS] = ns;
    }
    if (pass < 3) {   // the buffer the next pass counts into
        uint32_t *hn = qs + QS_BUF((pass + 1) % 3);
        for (uint32_t b = blockIdx.x * SKY_WG + t; b < P1 * SKY_HCOPY * 256; b += gridDim.x * SKY_WG) hn[b] = 0;
    }
    if (ns == 0) return;   // every selection settled (the same in every workgroup)
    for (uint32_t b = t; b < ns * 256; b += SKY_WG) h[b] = 0;
    __syncthreads();
    // row of each key: its prefix compared with every open one; none = 64
    uint32_t slot[QS_KPT];
#pragma unroll
    for (int k = 0; k < QS_KPT; ++k) slot[k] = pass == 0 && base + k * SKY_WG < n ? 0u : 64u;
    if (pass > 0)
        for (uint32_t q = 0; q < ns; ++q) {
            const uint32_t v = s_slotp[q];
#pragma unroll
            for (int k = 0; k < QS_KPT; ++k)
                if ((key[k] >> (shift + 8)) == v && base + k * SKY_WG < n) slot[k] = q;
        }
#pragma unroll
    for (int k = 0; k < QS_KPT; ++k)
        if (slot[k] < 64u) atomicAdd(&h[slot[k] * 256 + ((key[k] >> shift) & 255u)], 1u);
    __syncthreads();
    // read by the next launch: the kernel boundary orders it
    uint32_t *hc = qs + QS_BUF(pass % 3) + (blockIdx.x % SKY_HCOPY) * 256;
    for (uint32_t b = t; b < ns * 256; b += SKY_WG)
        if (h[b]) atomicAdd(&hc[(size_t)(b >> 8) * SKY_HCOPY * 256 + (b & 255u)], h[b]);
}

__global__ __launch_bounds__(SKY_WG) void k_qsel_pass(const float *__restrict__ xs, uint32_t n, int p, int pass,
                                                     uint32_t *qs, uint32_t *bnd, uint32_t *ctrl)
{
    extern __shared__ uint32_t h[];   // (p - 1) * 256
    qsel_pass_dev(xs, n, p, pass, qs, bnd, ctrl, h);
}

// qs: SKY_QSEL_WORDS words of workspace (row 0 of buffer 0 zero on entry);
// bnd: p - 1 words. 2 <= p <= SKY_QSEL_MAX_P. Four passes, then the last
// digit's step in one workgroup.
hipError_t launch_sliced_select(const float *xs, uint32_t n, int p, uint32_t *qs, uint32_t *bnd, uint32_t *ctrl,
                                hipStream_t s)
{
    if (n == 0 || p < 2 || p > SKY_QSEL_MAX_P) return hipErrorInvalidValue;
    const uint32_t per = QS_KPT * SKY_WG;
    const uint32_t blocks = (n + per - 1) / per;
    const size_t lds = (size_t)(p - 1) * 256 * 4;
    for (int pass = 0; pass < 5; ++pass)
        hipLaunchKernelGGL(k_qsel_pass, dim3(pass < 4 ? blocks : 1u), dim3(SKY_WG), lds, s, xs, n, p, pass, qs, bnd,
                           ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------------------ top-k select
// The k smallest points by (score, id) -- Sorted representatives take the
// coordinate sum, learned ones the MLP score (Section 4.1). MSB-first radix
// select over the unique 64-bit key (map(score) << 32 | id), 8 bits per pass.
// Up to two selections (two score arrays) run in the same passes: a histogram
// launch, then a one-workgroup pick of the digit that holds the k-th key.
// Selection state and histograms live in `sel` (uint32 words): three buffers of
// SKY_HCOPY copies of 512 words (pass t counts into buffer t % 3, copy b %
// SKY_HCOPY for workgroup b, and clears buffer (t + 1) % 3, which held the
// counts of pass t - 2; a bin's count is the sum of its copies), then two state sets of 8
// words, {k, prefix lo, prefix hi} of selection 1, then of selection 2, where
// k is the rank still to find (0: finished, the prefix is then the threshold).
// S_t, the state after pass t's digit, is computed by every workgroup of pass
// t + 1 and stored by its first one in set t & 1; pass t + 1 reads S_{t-1}
// from the other set, so no workgroup reads a set that is being written.
#define SEL_HIST(t) ((uint32_t)((t) % 3) * SKY_HCOPY * 512u)
#define SEL_STATE(t) (3u * SKY_HCOPY * 512u + (uint32_t)((t) & 1) * 8u)
#define SEL_KPT 16   // keys per thread and pass

// Digit position of a pass: passes 0..3 take the score's four bytes; the id
// passes take only the idd low bytes that an id below n can have (the higher
// id bytes are zero in every key and in every prefix), so a selection over n
// points has 4 + idd passes.
__device__ __forceinline__ int sel_shift(int pass, int idd)
{
    return pass < 4 ? 56 - 8 * pass : 8 * (idd + 3 - pass);
}
static int sel_id_digits(uint32_t n)
{
    int b = 1;
    while (b < 4 && (uint64_t)(n - 1) >> (8 * b)) ++b;
    return b;
}

struct SelState {
    uint32_t k;
    uint64_t prefix;
};

// The digit of one selection at `shift` from its 256-bin histogram (all 256
// threads call it; the result is uniform): the digit holding the k-th key
// extends the prefix; when every key with the extended prefix is needed, the
// selection is finished and its threshold is the prefix followed by all ones.
__device__ SelState sel_pick_state(const uint32_t *__restrict__ hist, SelState st, int shift, uint32_t *s_w,
                                   SelState *s_out)
{
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t v = 0;   // bin t: the sum of its copies
#pragma unroll
    for (int c = 0; c < SKY_HCOPY; ++c) v += hist[c * 512 + t];
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) s_w[wv] = x;
    __syncthreads();
    uint32_t base = 0;
    for (uint32_t w = 0; w < wv; ++w) base += s_w[w];
    const uint32_t incl = base + x, excl = incl - v;
    if (st.k && v && excl < st.k && st.k <= incl) {
        SelState r;
        r.prefix = st.prefix | ((uint64_t)t << shift);
        r.k = st.k - excl;
        if (r.k == v) {   // every key with this prefix is needed: done
            r.prefix |= (1ull << shift) - 1;
            r.k = 0;
        }
        *s_out = r;
    }
    __syncthreads();
    SelState r = st.k ? *s_out : st;
    __syncthreads();
    return r;
}

// S_{pass-1}, the state this pass selects by: pass 0 starts from (k1, 0),
// (k2, 0); pass t >= 1 picks the digits of pass t - 1 from S_{t-2} (the
// initial state for t = 1), and its first workgroup stores the result.
__device__ void sel_state(int pass, int idd, uint32_t k1, uint32_t k2, int two, uint32_t *sel, SelState &a,
                          SelState &b)
{
    __shared__ uint32_t s_w[4];
    __shared__ SelState s_out;
    a = SelState{k1, 0};
    b = SelState{two ? k2 : 0u, 0};
    if (pass == 0) return;
    if (pass > 1) {
        const uint32_t *st = sel + SEL_STATE(pass - 2);
        a = SelState{st[0], ((uint64_t)st[2] << 32) | st[1]};
        b = SelState{st[3], ((uint64_t)st[5] << 32) | st[4]};
    }
    const int shift = sel_shift(pass - 1, idd);
    const uint32_t *h = sel + SEL_HIST(pass - 1);
    a = sel_pick_state(h, a, shift, s_w, &s_out);
    if (two) b = sel_pick_state(h + 256, b, shift, s_w, &s_out);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        uint32_t *o = sel + SEL_STATE(pass - 1);
        o[0] = a.k; o[1] = (uint32_t)a.prefix; o[2] = (uint32_t)(a.prefix >> 32);
        o[3] = b.k; o[4] = (uint32_t)b.prefix; o[5] = (uint32_t)(b.prefix >> 32);
    }
}

// One pass: the previous pass's pick, then 256-bin histograms of the pass's
// digit over the keys that match the selected prefixes. A finished selection
// (k = 0) is skipped.
__global__ __launch_bounds__(SKY_WG) void k_sel_pass(const float *__restrict__ score,
                                                    const float *__restrict__ score2, uint32_t n, int pass, int idd,
                                                    uint32_t k1, uint32_t k2, uint32_t *sel, QselJob qj)
{
    static_assert(QS_KPT == SEL_KPT, "one grid for both selections");
    __shared__ uint32_t h[512];
    extern __shared__ uint32_t hq[];   // the Sliced selection's histograms, (p - 1) * 256 words
    if (qj.qs && (pass < 4 || (pass == 4 && blockIdx.x == 0)))   // pass 4: the last digit's step
        qsel_pass_dev(qj.xs, n, qj.p, pass, qj.qs, qj.bnd, qj.ctrl, hq);
    const uint32_t t = threadIdx.x, lane = t & 63;
    const int two = score2 != nullptr;
    if (pass >= 2) {   // finished before the previous pass: only carry the state over
        const uint32_t *st = sel + SEL_STATE(pass - 2);
        if (__builtin_amdgcn_readfirstlane(st[0]) == 0 && __builtin_amdgcn_readfirstlane(st[3]) == 0) {
            if (blockIdx.x == 0 && t < 8) sel[SEL_STATE(pass - 1) + t] = st[t];
            return;
        }
    }
    // this pass's keys first: their loads overlap the pick
    const uint32_t base = blockIdx.x * SKY_WG * SEL_KPT + t;
    uint32_t sc[SEL_KPT], sc2[SEL_KPT];
#pragma unroll
    for (int k = 0; k < SEL_KPT; ++k) {
        const uint32_t i = base + k * SKY_WG;
        sc[k] = i < n ? ordmap(score[i]) : 0xFFFFFFFFu;
        sc2[k] = (two && i < n) ? ordmap(score2[i]) : 0xFFFFFFFFu;
    }
    SelState a, b;
    sel_state(pass, idd, k1, k2, two, sel, a, b);
    if (blockIdx.x == 0)   // clear the buffer the next pass counts into
        for (uint32_t w = t; w < SKY_HCOPY * 512; w += SKY_WG) sel[SEL_HIST(pass + 1) + w] = 0;
    if (!a.k && !b.k) return;
    h[t] = 0;
    h[256 + t] = 0;
    __syncthreads();
    const int shift = sel_shift(pass, idd), hs = shift + 8;
#pragma unroll
    for (int k = 0; k < SEL_KPT; ++k) {
        const uint32_t i = base + k * SKY_WG;
        const bool in = i < n;
        for (int q = 0; q < 1 + two; ++q) {
            const SelState &st = q ? b : a;
            const uint64_t key = ((uint64_t)(q ? sc2[k] : sc[k]) << 32) | i;
            const bool m = in && st.k && (hs >= 64 || (key >> hs) == (st.prefix >> hs));
            const uint32_t dg = m ? (uint32_t)(key >> shift) & 255u : 256u;
            if (pass == 0) {
                // most keys share a few top digits: one LDS update per distinct digit in the wave
                uint64_t todo = __ballot(dg < 256u);
                while (todo) {
                    const uint32_t first = (uint32_t)__builtin_ctzll(todo);
                    const uint32_t v = __shfl(dg, (int)first, 64);
                    const uint64_t same = __ballot(dg == v);
                    if (lane == first) atomicAdd(&h[q * 256 + v], (uint32_t)__popcll(same));
                    todo &= ~same;
                }
            } else if (dg < 256u) {
                atomicAdd(&h[q * 256 + dg], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *hg = sel + SEL_HIST(pass) + (blockIdx.x % SKY_HCOPY) * 512;
    if (h[t]) atomicAdd(&hg[t], h[t]);
    if (h[256 + t]) atomicAdd(&hg[256 + t], h[256 + t]);
}

// The last pick, then the keys <= the thresholds: selection 1 into
// cand[0..SKY_MAXREPS), selection 2 into cand[SKY_MAXREPS ..]; counts in
// ctrl[C_NCAND], ctrl[C_NCAND2] (keys are unique, so at most k qualify).
__global__ __launch_bounds__(SKY_WG) void k_sel_collect(const float *__restrict__ score,
                                                       const float *__restrict__ score2, uint32_t n, int idd,
                                                       uint32_t k1, uint32_t k2, uint32_t *sel, uint32_t *ctrl,
                                                       uint64_t *cand)
{
    SelState a, b;
    const int two = score2 != nullptr;
    sel_state(4 + idd, idd, k1, k2, two, sel, a, b);
    const uint64_t thr = a.prefix, thr2 = b.prefix;
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        const uint64_t key = ((uint64_t)ordmap(score[i]) << 32) | i;
        if (key <= thr) {
            const uint32_t slot = atomicAdd(&ctrl[C_NCAND], 1u);
            if (slot < SKY_MAXREPS) cand[slot] = key;
        }
        if (two) {
            const uint64_t key2 = ((uint64_t)ordmap(score2[i]) << 32) | i;
            if (key2 <= thr2) {
                const uint32_t slot = atomicAdd(&ctrl[C_NCAND2], 1u);
                if (slot < SKY_MAXREPS) cand[SKY_MAXREPS + slot] = key2;
            }
        }
    }
}

// The k smallest points by (score, id) (and the k2 smallest by score2 in the
// same passes). sel: SKY_SEL_WORDS words, histogram buffer 0 zero on entry.
// qj (nullable): a Sliced boundary selection over the same n points, whose four
// passes run inside the first four select launches.
hipError_t launch_topk(const float *score, const float *score2, uint32_t n, int k, int k2, uint32_t *ctrl,
                       uint32_t *sel, uint64_t *cand, hipStream_t s, const QselJob *qj)
{
    if (qj && (qj->p < 2 || qj->p > SKY_QSEL_MAX_P)) return hipErrorInvalidValue;
    const QselJob q = qj ? *qj : QselJob{};
    const size_t lds = qj ? (size_t)(qj->p - 1) * 256 * 4 : 0;
    if (n == 0 || k <= 0 || k > SKY_MAXREPS || (score2 && (k2 <= 0 || k2 > SKY_MAXREPS)))
        return n == 0 ? hipSuccess : hipErrorInvalidValue;
    const uint32_t per = SEL_KPT * SKY_WG;
    const uint32_t blocks = (n + per - 1) / per;
    const int idd = sel_id_digits(n);   // 4 + idd >= 5 passes: the Sliced selection uses passes 0..4
    for (int pass = 0; pass < 4 + idd; ++pass)
        hipLaunchKernelGGL(k_sel_pass, dim3(blocks), dim3(SKY_WG), pass <= 4 ? lds : 0, s, score, score2, n, pass,
                           idd, (uint32_t)k, (uint32_t)k2, sel, q);
    uint32_t cb = (n + SKY_WG - 1) / SKY_WG;
    if (cb > 2048) cb = 2048;
    hipLaunchKernelGGL(k_sel_collect, dim3(cb), dim3(SKY_WG), 0, s, score, score2, n, idd, (uint32_t)k,
                       (uint32_t)k2, sel, ctrl, cand);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Sorted representatives per partition
// Section 4.1's Sorted strategy taken per partition: the kp = ceil(K / p)
// smallest points of every partition by (float32 sum, id), over all of its
// points. The keys (partition, mapped sum) are sorted stably with the ids as
// values (ids ascending, so equal keys keep id order); an entry whose run of
// equal partitions has fewer than kp entries before it becomes a candidate
// with key (partition * kp + offset) << 32 | id, which the finalize turns into
// partition-major order, each partition's in (sum, id) order.
__global__ __launch_bounds__(SKY_WG) void k_part_keys(const float *__restrict__ score,
                                                     const uint32_t *__restrict__ part, uint32_t n, uint64_t *keys,
                                                     uint32_t *vals)
{
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        keys[i] = ((uint64_t)part[i] << 32) | ordmap(score[i]);
        vals[i] = i;
    }
}

__global__ __launch_bounds__(SKY_WG) void k_part_picks(const uint64_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ vals, uint32_t n, uint32_t kp,
                                                      uint32_t *ctrl, uint64_t *cand)
{
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        const uint32_t pi = (uint32_t)(keys[i] >> 32);
        if (i >= kp && (uint32_t)(keys[i - kp] >> 32) == pi) continue;   // kp earlier entries in its partition
        uint32_t off = 0;
        while (off < i && (uint32_t)(keys[i - off - 1] >> 32) == pi) ++off;
        const uint32_t slot = atomicAdd(&ctrl[C_NCAND], 1u);
        if (slot < SKY_MAXREPS) cand[slot] = ((uint64_t)(pi * kp + off) << 32) | vals[i];
    }
}

hipError_t launch_part_reps(const float *score, const uint32_t *part, uint32_t n, int kp, int pbits, SortBufs &sb,
                            uint32_t *ctrl, uint64_t *cand, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_part_keys, dim3(blocks), dim3(SKY_WG), 0, s, score, part, n, sb.kA, sb.vA);
    hipError_t e = launch_radix_sort(sb, nullptr, n, 0, 32 + pbits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_part_picks, dim3(blocks), dim3(SKY_WG), 0, s, sb.kA, sb.vA, n, (uint32_t)kp, ctrl, cand);
    return hipGetLastError();
}

// ------------------------------------------------------------------ learned representatives
// Pool: cand[0 .. C_NCAND) are the smallest keys by coordinate sum and
// cand[SKY_MAXREPS ..] the smallest by learned score (at most SKY_POOL_HALF
// each, unordered). Pool slot j < SKY_POOL_HALF is the j-th sum candidate in
// key order, slot SKY_POOL_HALF + j the j-th learned one; a learned candidate
// already among the sum candidates, and unused slots, hold 0xFFFFFFFF.
//
// Mix choice: candidate set S_i (i = 0..4) holds the first R - m_i sum slots
// and the first m_i learned slots, m_i = floor(i*R/4), R = min(n_reps,
// SKY_POOL_HALF). S_i covers a point of the stride sample (input ids
// floor(s*n/M), s < M) when one of its slots dominates it (Def. 1 on the
// order-preserving images). The set that covers the most sample points wins
// (ties: the smaller i); its valid slots, sum part first, become the picks:
// picked[r] = (r << 32) | id, ctrl[C_NPICK] their count.
//
// One fused kernel. Every workgroup ranks the candidates itself (keys are
// distinct, so a key's rank is the count of smaller keys in its half) and
// loads the pool's coordinates into LDS. Workgroup g holds sample points
// 64g .. 64g+63, one per lane; wave v tests them against slots 32v .. 32v+31
// and keeps a 32-bit mask of the slots that dominate its lane's point. With
// the four masks of a lane joined into sum and learned halves, S_i covers the
// point iff a sum slot below R - m_i or a learned slot below m_i is set (an
// unused slot holds all-ones coordinates and dominates nothing). Per-set
// counts go to ctrl[C_MIX0 + i] (zeroed with ctrl); the workgroup that takes
// the last ticket of ctrl[C_MIXT] makes the choice. Workgroup 0 also stores
// the pool in pool_ids.
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_pool_mix(const float *__restrict__ pts, uint32_t n, int d, uint32_t M,
                                                    const uint64_t *__restrict__ cand, int n_reps, uint32_t *ctrl,
                                                    uint32_t *pool_ids, uint64_t *picked)
{
    constexpr int KD = DP - 2 < SKY_MAXD ? DP - 2 : SKY_MAXD;   // d <= KD
    constexpr uint32_t H = SKY_POOL_HALF, NW = SKY_WG / 64, SPW = 2 * H / NW;   // slots per wave
    static_assert(2 * H == SKY_WG / 2 && SPW == 32 && H == 64, "four waves of 32 slots");
    __shared__ uint64_t sk[2 * H];
    __shared__ uint32_t sid[2 * H];
    __shared__ __align__(16) uint32_t sp[KD][2 * H];   // pool coordinates, [k][slot]
    __shared__ uint32_t s_mask[NW][64];
    __shared__ uint32_t s_last;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t R = (uint32_t)min(n_reps, (int)H);

    // this lane's sample point, loaded first so that its latency overlaps the
    // pool set-up (coordinates past d repeat coordinate d - 1 and are unused)
    const uint32_t sidx = blockIdx.x * 64 + lane;
    const bool in = sidx < M;
    const uint32_t q = in ? (uint32_t)(((uint64_t)sidx * n) / M) : 0u;
    uint32_t c[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) c[k] = ordmap(pts[(size_t)min(k, d - 1) * n + q]);

    // pool slots
    const uint32_t half = t / H, j = t % H;
    if (t < 2 * H) {
        const uint32_t cnt = min(ctrl[half ? C_NCAND2 : C_NCAND], H);
        sk[t] = j < cnt ? cand[half * SKY_MAXREPS + j] : ~0ull;
    }
    __syncthreads();
    if (t < 2 * H) {
        const uint64_t key = sk[t];
        uint32_t rank = j;   // an unused entry keeps its place behind the used ones
        if (key != ~0ull) {
            rank = 0;
#pragma unroll 16
            for (uint32_t q = 0; q < H; ++q) rank += sk[half * H + q] < key ? 1u : 0u;
        }
        sid[half * H + rank] = key == ~0ull ? 0xFFFFFFFFu : (uint32_t)key;
    }
    __syncthreads();
    if (t >= H && t < 2 * H) {   // reads the sum half, writes only its own learned slot
        uint32_t id = sid[t];
        bool dup = false;
#pragma unroll 16
        for (uint32_t q = 0; q < H; ++q) dup = dup || sid[q] == id;
        sid[t] = dup ? 0xFFFFFFFFu : id;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t < 2 * H) pool_ids[t] = sid[t];
    {   // thread t loads coordinates k = t / 128, t / 128 + 2, .. of slot t % 128, all loads first
        const uint32_t slot = t % (2 * H), id = sid[slot];
        const uint32_t pid = id != 0xFFFFFFFFu ? id : 0u;
        uint32_t v[(KD + 1) / 2];
#pragma unroll
        for (int i = 0; i < (KD + 1) / 2; ++i) {
            const int k = 2 * i + (int)(t / (2 * H));
            v[i] = ordmap(pts[(size_t)min(k, d - 1) * n + pid]);
        }
#pragma unroll
        for (int i = 0; i < (KD + 1) / 2; ++i) {
            const int k = 2 * i + (int)(t / (2 * H));
            if (k < KD) sp[k][slot] = (id != 0xFFFFFFFFu && k < d) ? v[i] : 0xFFFFFFFFu;
        }
    }
    __syncthreads();

    // the sample point against this wave's 32 slots
    uint32_t fail = 0, less = 0;   // bit b: slot 32*wv + b exceeds / undercuts the point in some coordinate
#pragma unroll
    for (int k = 0; k < KD; ++k)
        if (k < d) {
            const uint32_t ck = c[k];
            const uint4 *row = reinterpret_cast<const uint4 *>(&sp[k][wv * SPW]);
#pragma unroll
            for (uint32_t b4 = 0; b4 < SPW / 4; ++b4) {
                const uint4 v = row[b4];
                fail |= (v.x > ck ? 1u : 0u) << (4 * b4) | (v.y > ck ? 1u : 0u) << (4 * b4 + 1) |
                        (v.z > ck ? 1u : 0u) << (4 * b4 + 2) | (v.w > ck ? 1u : 0u) << (4 * b4 + 3);
                less |= (v.x < ck ? 1u : 0u) << (4 * b4) | (v.y < ck ? 1u : 0u) << (4 * b4 + 1) |
                        (v.z < ck ? 1u : 0u) << (4 * b4 + 2) | (v.w < ck ? 1u : 0u) << (4 * b4 + 3);
            }
        }
    s_mask[wv][lane] = in ? (less & ~fail) : 0u;
    __syncthreads();
    if (wv == 0) {
        const uint64_t sum = (uint64_t)s_mask[0][lane] | (uint64_t)s_mask[1][lane] << 32;
        const uint64_t lrn = (uint64_t)s_mask[2][lane] | (uint64_t)s_mask[3][lane] << 32;
        for (uint32_t i = 0; i < 5; ++i) {
            const uint32_t mi = i * R / 4, ns = R - mi;
            const uint64_t ms = ns >= 64 ? ~0ull : (1ull << ns) - 1, ml = mi >= 64 ? ~0ull : (1ull << mi) - 1;
            const uint64_t bl = __ballot((sum & ms) != 0 || (lrn & ml) != 0);
            if (lane == 0) sky_consume(atomicAdd(&ctrl[C_MIX0 + i], (uint32_t)__popcll(bl)));
        }
    }
    __syncthreads();
    if (t == 0) s_last = atomicAdd(&ctrl[C_MIXT], 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    if (t == 0) {
        uint32_t best = 0, bc = 0;
        for (uint32_t i = 0; i < 5; ++i) {
            const uint32_t cv = atomicAdd(&ctrl[C_MIX0 + i], 0u);
            if (i == 0 || cv > bc) { best = i; bc = cv; }
        }
        const uint32_t ms = best * R / 4;
        uint32_t np_ = 0;
        for (uint32_t k = 0; k < R - ms; ++k)
            if (sid[k] != 0xFFFFFFFFu) { picked[np_] = ((uint64_t)np_ << 32) | sid[k]; ++np_; }
        for (uint32_t k = 0; k < ms; ++k)
            if (sid[H + k] != 0xFFFFFFFFu) { picked[np_] = ((uint64_t)np_ << 32) | sid[H + k]; ++np_; }
        ctrl[C_NPICK] = np_;
    }
}

hipError_t launch_pool_mix(const float *pts, uint32_t n, int d, const uint64_t *cand, uint32_t *ctrl,
                              uint32_t *pool_ids, int n_reps, uint64_t *picked, hipStream_t s)
{
    const uint32_t M = n < SKY_COVER_M ? n : SKY_COVER_M;
#define M_CASE(X)                                                                                         \
    case X:                                                                                               \
        hipLaunchKernelGGL(k_pool_mix<X>, dim3(SKY_COVER_M / 64), dim3(SKY_WG), 0, s, pts, n, d, M, cand, n_reps, \
                           ctrl, pool_ids, picked);                                                       \
        break;
    switch (sky_dp(d)) {
        M_CASE(4) M_CASE(8) M_CASE(12) M_CASE(16) M_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef M_CASE
    return hipGetLastError();
}

// Sort the (at most 256) candidates, build their records and apply the
// representative self-filter: a representative dominated by another one is
// discarded before the set is shared (Section 4.1). Kept records are
// compacted in score order into krec.
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_reps_finalize(const float *__restrict__ pts, uint32_t n, int d,
                                                         const uint64_t *__restrict__ cand, int count_slot,
                                                         uint32_t *ctrl, uint32_t *rep_ids, uint8_t *rep_keep,
                                                         uint32_t *krec)
{
    static_assert(SKY_MAXREPS == SKY_WG, "one thread per candidate");
    __shared__ uint64_t sk[SKY_MAXREPS];
    __shared__ __align__(16) uint32_t rec[SKY_MAXREPS * DP];
    __shared__ uint32_t sid[SKY_MAXREPS];
    __shared__ uint32_t s_tmp[4];
    const uint32_t t = threadIdx.x;
    uint32_t c = ctrl[count_slot];
    if (c > SKY_MAXREPS) c = SKY_MAXREPS;
    // candidate t's key and coordinates (all loads issued together; past d they
    // repeat coordinate d - 1 and are replaced by zero words)
    const uint64_t key = t < c ? cand[t] : ~0ull;
    const uint32_t cid = t < c ? (uint32_t)key : 0u;
    uint32_t w[DP - 2];
#pragma unroll
    for (int k = 0; k < DP - 2; ++k) w[k] = ordmap(pts[(size_t)min(k, d - 1) * n + cid]);
    sk[t] = key;
    __syncthreads();
    // score order: a key's rank is the count of smaller keys (keys are distinct)
    uint32_t rank = t;
    if (t < c) {
        rank = 0;
#pragma unroll 8
        for (uint32_t j = 0; j < c; ++j) rank += sk[j] < key ? 1u : 0u;
        uint64_t K = 0;
#pragma unroll
        for (int k = 0; k < DP - 2; ++k) {
            if (k >= d) w[k] = 0u;
            rec[rank * DP + k] = w[k];
            K += w[k];
        }
        rec[rank * DP + DP - 2] = (uint32_t)K;
        rec[rank * DP + DP - 1] = (uint32_t)(K >> 32);
        sid[rank] = cid;
    }
    __syncthreads();
    // self-filter of representative t (in score order) against all others;
    // every thread reads the same record j, so the LDS reads broadcast. A whole
    // record per step and no branches, so the reads of several steps are in
    // flight together (the words past d are zero on both sides).
    const uint32_t id = sid[t];
    bool keep = t < c;
    if (keep) {
        uint32_t my[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) my[k] = rec[t * DP + k];
        uint32_t dominated = 0;
#pragma unroll 4
        for (uint32_t j = 0; j < c; ++j) {
            const uint4 *rj = reinterpret_cast<const uint4 *>(rec + j * DP);
            uint32_t o[DP];
#pragma unroll
            for (int k4 = 0; k4 < DP / 4; ++k4) {
                const uint4 v = rj[k4];
                o[4 * k4] = v.x; o[4 * k4 + 1] = v.y; o[4 * k4 + 2] = v.z; o[4 * k4 + 3] = v.w;
            }
            uint32_t dm = j != t ? 1u : 0u;
#pragma unroll
            for (int k = 0; k < DP - 2; ++k) dm &= o[k] <= my[k] ? 1u : 0u;
            dm &= ((o[DP - 2] != my[DP - 2]) | (o[DP - 1] != my[DP - 1])) ? 1u : 0u;
            dominated |= dm;
        }
        keep = dominated == 0;
    }
    uint32_t tot;
    const int lane = t & 63, wv = t >> 6;
    const uint64_t m = __ballot(keep);
    if (lane == 0) s_tmp[wv] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t r = (uint32_t)__popcll(m & lmask_lt());
    for (int w = 0; w < wv; ++w) r += s_tmp[w];
    tot = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    if (keep)
        for (int k = 0; k < DP; ++k) krec[r * DP + k] = rec[t * DP + k];
    // pad to a multiple of 4 records with all-ones coordinates, which no
    // finite point's mapped coordinates reach, so a pad dominates nothing
    if (t >= tot && t < ((tot + 3u) & ~3u))
        for (int k = 0; k < DP; ++k) krec[t * DP + k] = 0xFFFFFFFFu;
    if (t < c) {
        rep_ids[t] = id;
        rep_keep[t] = keep ? 1 : 0;
    }
    if (t == 0) {
        ctrl[C_NREPS] = c;
        ctrl[C_NREPS_KEPT] = tot;
    }
}

hipError_t launch_reps_finalize(const float *pts, uint32_t n, int d, const uint64_t *cand, int count_slot,
                                uint32_t *ctrl, uint32_t *rep_ids, uint8_t *rep_keep, uint32_t *krec,
                                hipStream_t s)
{
    const int DP = sky_dp(d);
#define R_CASE(X)                                                                                     \
    case X:                                                                                           \
        hipLaunchKernelGGL(k_reps_finalize<X>, dim3(1), dim3(SKY_WG), 0, s, pts, n, d, cand, count_slot, \
                           ctrl, rep_ids, rep_keep, krec);                                            \
        break;
    switch (DP) {
        R_CASE(4) R_CASE(8) R_CASE(12) R_CASE(16) R_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef R_CASE
    return hipGetLastError();
}

// Workgroups of the filter kernel (4 points per thread), also the length of its per-workgroup counts.
static uint32_t filter_blocks(uint32_t n)
{
    uint32_t blocks = (n + 4 * SKY_WG - 1) / (4 * SKY_WG);
    return blocks > 4096 ? 4096 : blocks;
}

// ------------------------------------------------------------------ filter + partition id
// Per point: Grid Filtering (its cell is grid-dominated by a non-empty cell),
// Representative Filtering (a kept representative dominates it; the test is
// exact, so a representative never removes itself or its duplicates), and the
// Grid or Angular partition id.
//  Grid (Section 3.2): id = sum_k floor(x_k m_k) prod_{j<k} m_j, clamped.
//  Angular (Section 3.3, Eq. (1)): the digit of angle a counts the k in
//  1..m_a-1 with S_a >= x_a^2 T[a][k], S_a = sum_{j>a} x_j^2, T = tan^2(k pi/(2 m_a)),
//  all in float64 with explicit round-to-nearest operations in index order.
template <int DP, int NC>
__global__ __launch_bounds__(SKY_WG) void k_filter(const float *__restrict__ pts, uint32_t n, int d,
                                                  int gf_on, GridSpec gg, const uint32_t *__restrict__ gdom,
                                                  int use_reps, const uint32_t *__restrict__ krec,
                                                  int part_kind, GridSpec pg, AngSpec ag,
                                                  const uint32_t *__restrict__ sbnd, int sdim,
                                                  uint32_t *__restrict__ part, uint32_t *part_hist, int np,
                                                  uint8_t *__restrict__ alive, uint32_t *ctrl, uint32_t *grid_cnt)
{
    // points per thread: each representative load serves FPP * 256 points;
    // fewer for wider records, whose coordinates would spill registers
    constexpr int ND = DP - 2, FPP = DP <= 4 ? 4 : DP <= 16 ? 2 : 1;
    __shared__ uint32_t s_hist[4096];
    const uint32_t nk = use_reps ? __builtin_amdgcn_readfirstlane(ctrl[C_NREPS_KEPT]) : 0u;
    const bool lds_hist = (part_kind == P_GRID || part_kind == P_ANGULAR) && np <= 4096;
    if (lds_hist)
        for (int i = threadIdx.x; i < np; i += SKY_WG) s_hist[i] = 0;
    __syncthreads();
    uint32_t cnt_grid = 0;
    for (uint32_t base = blockIdx.x * SKY_WG * FPP; base < n; base += gridDim.x * SKY_WG * FPP) {
        float x[FPP][ND];
        uint32_t w[FPP][ND];
        uint64_t K[FPP];
        bool a[FPP];
#pragma unroll
        for (int q = 0; q < FPP; ++q) {
            const uint32_t i = base + q * SKY_WG + threadIdx.x;
            const uint32_t ii = i < n ? i : n - 1;
#pragma unroll
            for (int k = 0; k < ND; ++k) x[q][k] = k < d ? pts[(size_t)k * n + ii] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < FPP; ++q) {
            const uint32_t i = base + q * SKY_WG + threadIdx.x;
            K[q] = 0;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                w[q][k] = (k < d) ? ordmap(x[q][k]) : 0u;
                K[q] += w[q][k];
            }
            a[q] = i < n;
            if (gf_on && a[q]) {
                uint32_t cell = 0, mult = 1;
                for (int k = 0; k < d; ++k) {
                    cell += grid_digit(x[q][k], gg.m[k]) * mult;
                    mult *= (uint32_t)gg.m[k];
                }
                if ((gdom[cell >> 5] >> (cell & 31)) & 1u) a[q] = false;
            }
            cnt_grid += a[q] ? 1u : 0u;
        }
        // representatives: read-only, wave-uniform records -> scalar loads, scalar operands;
        // four records per batch, their loads issued together. The four points of a
        // lane are four rows of the wave's live masks, tested as the dominance kernels
        // test query rows.
        if (nk) {
            uint64_t am[FPP];
#pragma unroll
            for (int q = 0; q < FPP; ++q) am[q] = __ballot(a[q]);
            const uint32_t *rp = krec;
            // no early exit once every row is dead: a loop with a second exit gets vector
            // record loads from the compiler (measured slower than the 16 batches at most)
            for (uint32_t r = 0; r < nk; r += 4, rp += 4 * DP) {
                uint32_t rr[4][DP];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int k = 0; k < DP; ++k) rr[u][k] = rp[u * DP + k];
#pragma unroll
                for (int u = 0; u < 4; ++u) test_rec<DP, NC, FPP>(rr[u], w, K, am);
            }
            const uint32_t lane = threadIdx.x & 63;
#pragma unroll
            for (int q = 0; q < FPP; ++q) a[q] = (am[q] >> lane) & 1ull;
        }
#pragma unroll
        for (int q = 0; q < FPP; ++q) {
            const uint32_t i = base + q * SKY_WG + threadIdx.x;
            if (i >= n) continue;
            uint32_t pid = 0;
            if (part_kind == P_GRID) {
                uint32_t mult = 1;
                for (int k = 0; k < d; ++k) {
                    pid += grid_digit(x[q][k], pg.m[k]) * mult;
                    mult *= (uint32_t)pg.m[k];
                }
            } else if (part_kind == P_ANGULAR) {
                uint32_t mult = 1;
                for (int a2 = 0; a2 < d - 1; ++a2) {
                    double S = 0.0;
                    for (int j = a2 + 1; j < d; ++j) {
                        const double xj = (double)x[q][j];
                        S = __dadd_rn(S, __dmul_rn(xj, xj));
                    }
                    const double xi = (double)x[q][a2];
                    const double x2 = __dmul_rn(xi, xi);
                    uint32_t digit = 0;
                    for (int k = 1; k < ag.m[a2]; ++k)
                        if (S >= __dmul_rn(x2, ag.T[a2][k])) digit = (uint32_t)k;
                    pid += digit * mult;
                    mult *= (uint32_t)ag.m[a2];
                }
            } else if (part_kind == P_SLICED && sbnd) {   // slice = number of boundary keys <= map(x_s)
                uint32_t ks = 0;
#pragma unroll
                for (int k = 0; k < ND; ++k)
                    if (k == sdim) ks = w[q][k];
                for (int j = 0; j < np - 1; ++j) pid += ks >= sbnd[j] ? 1u : 0u;
                part[i] = pid;
            }
            if (part_kind == P_GRID || part_kind == P_ANGULAR) {
                part[i] = pid;
                if (lds_hist) atomicAdd(&s_hist[pid], 1u);
                else atomicAdd(&part_hist[pid], 1u);
            }
            alive[i] = a[q] ? 1 : 0;
        }
    }
    // per-workgroup count of grid survivors (summed later; a global atomic per
    // wave on one address would serialise)
    for (int o = 32; o > 0; o >>= 1) cnt_grid += __shfl_xor(cnt_grid, o, 64);
    __shared__ uint32_t s_cnt[4];
    if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt_grid;
    __syncthreads();
    if (threadIdx.x == 0) grid_cnt[blockIdx.x] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    if (lds_hist) {
        __syncthreads();
        for (int j = threadIdx.x; j < np; j += SKY_WG)
            if (s_hist[j]) atomicAdd(&part_hist[j], s_hist[j]);
    }
}

hipError_t launch_filter(const float *pts, uint32_t n, int d, int gf_on, const GridSpec &gg,
                         const uint32_t *gdom, int use_reps, const uint32_t *krec, int part_kind,
                         const GridSpec &pg, const AngSpec &ag, const uint32_t *sbnd, int sdim, uint32_t *part,
                         uint32_t *part_hist, int np, uint8_t *alive, uint32_t *ctrl, uint32_t *grid_cnt,
                         hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint32_t blocks = filter_blocks(n);   // every block writes its grid_cnt entry
    const int DP = sky_dp(d), NC = sky_nc(d);
#define F_CASE(X, C)                                                                                        \
    case X * 32 + C:                                                                                        \
        hipLaunchKernelGGL((k_filter<X, C>), dim3(blocks), dim3(SKY_WG), 0, s, pts, n, d, gf_on, gg, gdom, \
                           use_reps, krec, part_kind, pg, ag, sbnd, sdim, part, part_hist, np, alive, ctrl,  \
                           grid_cnt);                                                                       \
        break;
    switch (DP * 32 + NC) {
        F_CASE(4, 2) F_CASE(8, 4) F_CASE(8, 6) F_CASE(12, 8) F_CASE(12, 10) F_CASE(16, 12) F_CASE(16, 14)
        F_CASE(20, 16)
        default: return hipErrorInvalidValue;
    }
#undef F_CASE
    return hipGetLastError();
}

// Sum of the per-workgroup grid-survivor counts into ctrl[C_NGRID].
__global__ __launch_bounds__(SKY_WG) void k_sum_grid(const uint32_t *__restrict__ cnt, uint32_t nblk, uint32_t *ctrl)
{
    __shared__ uint32_t s_w[4];
    uint32_t a = 0;
    for (uint32_t i = threadIdx.x; i < nblk; i += SKY_WG) a += cnt[i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) ctrl[C_NGRID] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

hipError_t launch_sum_grid(const uint32_t *grid_cnt, uint32_t n, uint32_t *ctrl, hipStream_t s)
{
    const uint32_t blocks = n == 0 ? 0u : filter_blocks(n);
    hipLaunchKernelGGL(k_sum_grid, dim3(1), dim3(SKY_WG), 0, s, grid_cnt, blocks, ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Region and random choices
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) in counter form: draw i from
// state seed is the generator's output for state seed + (i + 1) * gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

#define REPS_STREAM 0xD1B54A32D192ED03ull   // the representatives' draws use seed ^ this word

// Region (Section 4.1): -V with V = prod_k (1 - x_k), the volume of the
// dominance region on [0,1]^d, multiplied in coordinate order in float32 (the
// range is checked by the ingest). Random: a uniform score on the 2^-24 grid.
// The representatives are the n_reps smallest scores (ties by id).
__global__ __launch_bounds__(SKY_WG) void k_rep_scores(const float *__restrict__ pts, uint32_t n, int d, int kind,
                                                      uint64_t seed, float *__restrict__ score)
{
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        if (kind == 3) {
            float v = 1.0f;
            for (int k = 0; k < d; ++k) v = v * (1.0f - pts[(size_t)k * n + i]);
            score[i] = -v;
        } else {
            score[i] = (float)(splitmix64(seed ^ REPS_STREAM, i) >> 40) * 0x1p-24f;
        }
    }
}

hipError_t launch_rep_scores(const float *pts, uint32_t n, int d, int kind, uint64_t seed, float *score,
                             hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (kind != 3 && kind != 4) return hipErrorInvalidValue;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_rep_scores, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, d, kind, seed, score);
    return hipGetLastError();
}

// Random partitioning (Section 3.1): keys floor(h_i / 2^32) with values i; a
// stable sort of them ranks the points by (key, i), and rank r goes to
// partition floor(r p / n): equal-sized partitions of a random permutation.
__global__ __launch_bounds__(SKY_WG) void k_random_init(uint32_t n, uint64_t seed, uint64_t *keys, uint32_t *vals)
{
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        keys[i] = splitmix64(seed, i) >> 32;
        vals[i] = i;
    }
}

hipError_t launch_random_init(uint32_t n, uint64_t seed, uint64_t *keys, uint32_t *vals, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_random_init, dim3(blocks), dim3(SKY_WG), 0, s, n, seed, keys, vals);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Sliced partitioning
// Rank of every point in the order (x_s, then the other coordinates, then id),
// a total order and a linear extension of dominance; rank r goes to slice
// floor(r p / N) (Section 3.4). The ranks come from a stable sort by x_s
// alone (ties then stay in id order); if a run of equal x_s straddles a slice
// boundary, the points of such runs are re-sorted lexicographically (the tie
// refinement below) and written back over the runs' positions.
__global__ __launch_bounds__(SKY_WG) void k_sliced_init(const float *__restrict__ pts, uint32_t n, int coord,
                                                       uint64_t *keys, uint32_t *vals)
{
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        vals[i] = i;
        keys[i] = ordmap(pts[(size_t)coord * n + i]);
    }
}

hipError_t launch_sliced_init(const float *pts, uint32_t n, int coord, uint64_t *keys, uint32_t *vals,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_sliced_init, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, coord, keys, vals);
    return hipGetLastError();
}

__global__ __launch_bounds__(SKY_WG) void k_sliced_check(const uint64_t *__restrict__ keys, uint32_t n, int p,
                                                        uint32_t *ctrl)
{
    for (int j = 1 + threadIdx.x; j < p; j += SKY_WG) {
        const uint64_t r = ((uint64_t)j * n + p - 1) / p;   // first rank of slice j
        if (r >= 1 && r < n && keys[r - 1] == keys[r]) atomicOr(&ctrl[C_TIE], 1u);
    }
}

__global__ __launch_bounds__(SKY_WG) void k_sliced_assign(const uint32_t *__restrict__ vals, uint32_t n, int p,
                                                         uint32_t *part)
{
    for (uint32_t r = blockIdx.x * SKY_WG + threadIdx.x; r < n; r += gridDim.x * SKY_WG)
        part[vals[r]] = (uint32_t)(((uint64_t)r * (uint64_t)p) / n);
}

hipError_t launch_sliced_check(const uint64_t *keys, uint32_t n, int p, uint32_t *ctrl, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sliced_check, dim3(1), dim3(SKY_WG), 0, s, keys, n, p, ctrl);
    return hipGetLastError();
}

hipError_t launch_sliced_assign(const uint32_t *vals, uint32_t n, int p, uint32_t *part, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_sliced_assign, dim3(blocks), dim3(SKY_WG), 0, s, vals, n, p, part);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Sliced tie refinement
// After the stable sort by (instance, x_s) from index order, only a run of equal
// keys that straddles a slice boundary needs the lexicographic order of the
// rest (the other coordinates in index order, then the index): every other
// point's rank is already final. The straddling runs' positions are marked,
// compacted, the subset is sorted on its own (LSD over the coordinates, then
// the run key) and written back over the same positions, which the runs fill
// in the same key order.

// Boundaries q = (instance i, slice j >= 1), grid-stride over workgroups: a run
// that straddles rank r_j of instance i is found by binary search in the
// instance's sorted keys and its positions [a, b) are flagged.
__global__ __launch_bounds__(SKY_WG) void k_tie_mark(const uint64_t *__restrict__ keys,
                                                    const uint32_t *__restrict__ goff, int ng, int p,
                                                    uint8_t *__restrict__ flag)
{
    const uint32_t nb = (uint32_t)ng * (uint32_t)(p - 1);
    for (uint32_t q = blockIdx.x; q < nb; q += gridDim.x) {
        const uint32_t i = q / (uint32_t)(p - 1), j = q % (uint32_t)(p - 1) + 1;
        const uint32_t g0 = goff[i], ni = goff[i + 1] - g0;
        const uint64_t r = ((uint64_t)j * ni + p - 1) / p;   // first rank of slice j
        if (r < 1 || r >= ni) continue;
        const uint32_t pos = g0 + (uint32_t)r;
        const uint64_t kv = keys[pos];
        if (keys[pos - 1] != kv) continue;
        uint32_t lo = g0, hi = pos;   // first position holding kv
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (keys[mid] < kv) lo = mid + 1; else hi = mid;
        }
        const uint32_t a = lo;
        lo = pos;
        hi = g0 + ni;   // first position past the run
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (keys[mid] <= kv) lo = mid + 1; else hi = mid;
        }
        for (uint32_t x = a + threadIdx.x; x < lo; x += SKY_WG) flag[x] = 1;
    }
}

// Flagged positions per segment of 1024 (one wave per segment).
#define TIE_SEG 1024
__global__ __launch_bounds__(SKY_WG) void k_tie_count(const uint8_t *__restrict__ flag, uint32_t n, uint32_t nseg,
                                                     uint32_t *cnt)
{
    const uint32_t lane = threadIdx.x & 63, sgi = blockIdx.x * (SKY_WG / 64) + (threadIdx.x >> 6);
    if (sgi < nseg) {
        const uint32_t b0 = sgi * TIE_SEG, e0 = min(n, b0 + TIE_SEG);
        uint32_t c = 0;
        for (uint32_t x = b0 + lane; x < e0; x += 64) c += flag[x] ? 1u : 0u;
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) cnt[sgi] = c;
    }
}

// The flagged positions in ascending order (pos_out) and the values there.
__global__ __launch_bounds__(SKY_WG) void k_tie_write(const uint8_t *__restrict__ flag, uint32_t n, uint32_t nseg,
                                                     const uint32_t *__restrict__ cnt,
                                                     const uint32_t *__restrict__ vals, uint32_t *pos_out,
                                                     uint32_t *vals_out)
{
    const uint32_t lane = threadIdx.x & 63, sgi = blockIdx.x * (SKY_WG / 64) + (threadIdx.x >> 6);
    if (sgi >= nseg) return;
    const uint32_t b0 = sgi * TIE_SEG, e0 = min(n, b0 + TIE_SEG);
    uint32_t o = cnt[sgi];
    for (uint32_t x0 = b0; x0 < e0; x0 += 64) {
        const uint32_t x = x0 + lane;
        const bool f = x < e0 && flag[x];
        const uint64_t m = __ballot(f);
        if (f) {
            const uint32_t t = o + (uint32_t)__popcll(m & ((1ull << lane) - 1));
            pos_out[t] = x;
            vals_out[t] = vals[x];
        }
        o += (uint32_t)__popcll(m);
    }
}

// keys[t] = map(x_coord) of point vals[t] (t < *m), above it the point's
// instance when inst is given.
__global__ __launch_bounds__(SKY_WG) void k_tie_rekey(const float *__restrict__ pts, uint32_t n, int coord,
                                                     const uint32_t *__restrict__ inst, const uint32_t *m_dev,
                                                     uint64_t *keys, const uint32_t *__restrict__ vals)
{
    const uint32_t m = *m_dev;
    for (uint32_t t = blockIdx.x * SKY_WG + threadIdx.x; t < m; t += gridDim.x * SKY_WG) {
        const uint32_t gi = vals[t];
        const uint64_t x = ordmap(pts[(size_t)coord * n + gi]);
        keys[t] = inst ? ((uint64_t)inst[gi] << 32) | x : x;
    }
}

// out[pos[t]] = vals[t] for t < *m.
__global__ __launch_bounds__(SKY_WG) void k_tie_back(const uint32_t *__restrict__ pos,
                                                    const uint32_t *__restrict__ vals, const uint32_t *m_dev,
                                                    uint32_t *out)
{
    const uint32_t m = *m_dev;
    for (uint32_t t = blockIdx.x * SKY_WG + threadIdx.x; t < m; t += gridDim.x * SKY_WG) out[pos[t]] = vals[t];
}

// Lexicographic refinement of the runs that straddle slice boundaries. In:
// b.kA / b.vA the (instance, x_s)-sorted keys and point indices (n of them,
// instance i at [goff[i], goff[i+1]), goff on the device), inst the point's
// instance (nullptr: one instance). Out: order[] = the refined point order.
// flag: n bytes of scratch (zero on entry); cnt: ceil(n / 1024) words; pos: n
// words. The coordinates other than sdim are the refinement keys, from d - 1
// down; the last sort is by the run key ((instance, x_s)), kbits wide.
#define TIE_TRY(x)                              \
    do {                                        \
        const hipError_t e_ = (x);              \
        if (e_ != hipSuccess) return e_;        \
    } while (0)
hipError_t launch_tie_refine(SortBufs &b, const float *pts, uint32_t n, int d, int sdim, const uint32_t *inst,
                             const uint32_t *goff, int ng, int p, int kbits, uint8_t *flag, uint32_t *cnt,
                             uint32_t *pos, uint32_t *order, uint32_t *ctrl, hipStream_t s)
{
    if (n == 0 || p < 2) return hipSuccess;
    TIE_TRY(hipMemcpyAsync(order, b.vA, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    const uint32_t nb = (uint32_t)ng * (uint32_t)(p - 1);
    hipLaunchKernelGGL(k_tie_mark, dim3(nb < 8192 ? nb : 8192), dim3(SKY_WG), 0, s, b.kA, goff, ng, p, flag);
    const uint32_t nseg = (n + TIE_SEG - 1) / TIE_SEG;
    const uint32_t cg = (nseg + SKY_WG / 64 - 1) / (SKY_WG / 64);
    hipLaunchKernelGGL(k_tie_count, dim3(cg), dim3(SKY_WG), 0, s, flag, n, nseg, cnt);
    TIE_TRY(launch_scan_counts(cnt, nseg, nullptr, ctrl + C_NTIE, s));   // ctrl[C_NTIE]: the subset's size
    hipLaunchKernelGGL(k_tie_write, dim3(cg), dim3(SKY_WG), 0, s, flag, n, nseg, cnt, order, pos, b.vA);
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 8192) blocks = 8192;
    const uint32_t *m = ctrl + C_NTIE;
    for (int k = d - 1; k >= 0; --k) {
        if (k == sdim) continue;
        hipLaunchKernelGGL(k_tie_rekey, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, k, (const uint32_t *)nullptr, m,
                           b.kA, b.vA);
        TIE_TRY(launch_radix_sort(b, m, n, 0, 32, s));
    }
    hipLaunchKernelGGL(k_tie_rekey, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, sdim, inst, m, b.kA, b.vA);
    TIE_TRY(launch_radix_sort(b, m, n, 0, kbits, s));
    hipLaunchKernelGGL(k_tie_back, dim3(blocks), dim3(SKY_WG), 0, s, pos, b.vA, m, order);
    return hipGetLastError();
}
#undef TIE_TRY

// ------------------------------------------------------------------ chunk table
// Partition j's points [poff[j], poff[j+1]) are cut into query groups of B
// points; nch[j] = their number and st_off the exclusive scan (group c of
// partition j is number st_off[j] + c). ctrl[which] = total groups, ctrl[C_MAXC]
// = the largest nch. One workgroup: thread t owns a contiguous range of
// partitions, so a single block scan suffices. With gpart (np <= CT_FUSE_NP,
// at most CT_FUSE_G groups) the same workgroup also writes the group map of
// k_group_part from copies of st_off and xoff in LDS: one launch instead of two.
// With urank as well, the workgroup first derives the offsets of the union of
// the local skylines, as k_union_offsets does (poff then holds the partitions'
// offsets; upoff, local_sizes and ctrl[C_MAXU] are written), and builds the
// table over those.
__global__ __launch_bounds__(1024) void k_chunk_table(const uint32_t *__restrict__ poff, int np, int B,
                                                      uint32_t *nch, uint32_t *st_off, uint32_t *ctrl, int which,
                                                      uint32_t *xoff, uint32_t *gpart, uint32_t *xlist,
                                                      const uint32_t *__restrict__ urank, const uint32_t *n_dev,
                                                      uint32_t *upoff, int64_t *local_sizes)
{
    __shared__ uint32_t s_w[16], s_m[16];
    __shared__ uint32_t s_st[CT_FUSE_NP + 1], s_xo[CT_FUSE_NP], s_up[CT_FUSE_NP + 1];
    const bool fuse = gpart != nullptr, uni = urank != nullptr;   // uni implies fuse (np <= CT_FUSE_NP)
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (uni) {
        const uint32_t n = *n_dev, nu = ctrl[C_NU];
        for (uint32_t j = t; j <= (uint32_t)np; j += 1024) {
            const uint32_t pj = poff[j];
            const uint32_t v = pj < n ? urank[pj] : nu;
            s_up[j] = v;
            upoff[j] = v;
        }
        __syncthreads();
        uint32_t mu = 0;
        for (uint32_t j = t; j < (uint32_t)np; j += 1024) {
            const uint32_t sz = s_up[j + 1] - s_up[j];
            mu = max(mu, sz);
            if (local_sizes) local_sizes[j] = (int64_t)sz;
        }
        for (int o = 32; o > 0; o >>= 1) mu = max(mu, (uint32_t)__shfl_xor((int)mu, o, 64));
        if (lane == 0) s_m[wv] = mu;
        __syncthreads();
        if (t == 0) {
            uint32_t m = 0;
            for (int w = 0; w < 16; ++w) m = max(m, s_m[w]);
            ctrl[C_MAXU] = m;
        }
        __syncthreads();   // s_m is reused below
    }
    // groups of partition j (offsets from LDS when the union's were derived here)
    auto groups_of = [&](uint32_t j) -> uint32_t {
        const uint32_t lo = uni ? s_up[j] : poff[j], hi = uni ? s_up[j + 1] : poff[j + 1];
        return (hi - lo + B - 1) / B;
    };
    const uint32_t per = ((uint32_t)np + 1023) / 1024;
    const uint32_t j0 = min((uint32_t)np, t * per), j1 = min((uint32_t)np, j0 + per);
    uint32_t sum = 0, mx = 0;
    for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t c = groups_of(j);
        sum += c;
        mx = max(mx, c);
    }
    uint32_t inc = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o) inc += v;
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if (lane == 63) s_w[wv] = inc;
    if (lane == 0) s_m[wv] = mx;
    __syncthreads();
    uint32_t run = inc - sum, tot = 0, M = 0;
    for (uint32_t w = 0; w < 16; ++w) {
        if (w < wv) run += s_w[w];
        tot += s_w[w];
        M = max(M, s_m[w]);
    }
    for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t c = groups_of(j);
        nch[j] = c;
        st_off[j] = run;
        if (fuse) s_st[j] = run;
        run += c;
    }
    if (t == 0) {
        st_off[np] = tot;
        ctrl[which] = tot;
        ctrl[C_MAXC] = M;
    }
    if (xoff) {
        // partition j belongs to XCD j % SKY_NXCD; ctrl[C_XG0 + x] = groups of XCD
        // x, and xoff[j] = where partition j's groups start in the XCD-major list
        // (thread x < 8 walks its partitions; used with np <= SKY_XCD_MAX_NP)
        __shared__ uint32_t s_xg[SKY_NXCD];
        __syncthreads();
        // (group counts recomputed from poff rather than read back from nch)
        if (t < SKY_NXCD) {
            uint32_t c = 0;
            for (uint32_t j = t; j < (uint32_t)np; j += SKY_NXCD) c += groups_of(j);
            s_xg[t] = c;
            ctrl[C_XG0 + t] = c;
        }
        __syncthreads();
        if (t < SKY_NXCD) {
            uint32_t pos = 0;
            for (uint32_t y = 0; y < t; ++y) pos += s_xg[y];
            for (uint32_t j = t; j < (uint32_t)np; j += SKY_NXCD) {
                xoff[j] = pos;
                if (fuse) s_xo[j] = pos;
                pos += groups_of(j);
            }
        }
    }
    if (!fuse) return;
    __syncthreads();
    // the group map (as k_group_part), tot groups in all
    for (uint32_t g = t; g < tot; g += 1024) {
        int lo = 0, hi = np - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_st[mid] <= g) lo = mid; else hi = mid - 1;
        }
        gpart[g] = (uint32_t)lo;
        if (xlist) xlist[s_xo[lo] + (g - s_st[lo])] = g;
    }
}

// gpart[g] = the partition of query group g (largest j with st_off[j] <= g).
// With xlist: the groups of each XCD's partitions listed XCD by XCD, each
// XCD's in partition order (xoff from the chunk table).
__global__ __launch_bounds__(SKY_WG) void k_group_part(const uint32_t *__restrict__ st_off,
                                                      const uint32_t *__restrict__ xoff, int np,
                                                      const uint32_t *ctrl, int which, uint32_t *gpart,
                                                      uint32_t *xlist)
{
    const uint32_t G = ctrl[which];
    for (uint32_t g = blockIdx.x * SKY_WG + threadIdx.x; g < G; g += gridDim.x * SKY_WG) {
        int lo = 0, hi = np - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (st_off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        gpart[g] = (uint32_t)lo;
        if (xlist) xlist[xoff[lo] + (g - st_off[lo])] = g;
    }
}

hipError_t launch_chunk_table(const uint32_t *poff, int np, int B, uint32_t *nch, uint32_t *st_off, uint32_t *gpart,
                              uint32_t *ctrl, int which, uint32_t g_max, hipStream_t s, uint32_t *xlist,
                              const UnionOffsets *u)
{
    if (np > SKY_XCD_MAX_NP) xlist = nullptr;
    uint32_t *xoff = xlist ? xlist + g_max : nullptr;   // np words after the list
    const bool fuse = chunk_table_fuses(np, g_max);
    if (u && !fuse) return hipErrorInvalidValue;
    if (fuse) {   // one workgroup writes the group map too
        hipLaunchKernelGGL(k_chunk_table, dim3(1), dim3(1024), 0, s, poff, np, B, nch, st_off, ctrl, which, xoff,
                           gpart, xlist, u ? u->urank : nullptr, u ? u->n_dev : nullptr, u ? u->upoff : nullptr,
                           u ? u->local_sizes : nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_chunk_table, dim3(1), dim3(1024), 0, s, poff, np, B, nch, st_off, ctrl, which, xoff,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    uint32_t blocks = (g_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_group_part, dim3(blocks), dim3(SKY_WG), 0, s, st_off, xoff, np, ctrl, which, gpart, xlist);
    return hipGetLastError();
}
