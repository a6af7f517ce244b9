// Skyline kernels for gfx950: ingest and validation, Grid Filtering,
// representative selection and filtering, partition assignment, the local
// skyline (SFS semantics) and the NoSeq merge.
//
// Dominance (Def. 1) is evaluated on order-preserving uint32 images of the
// coordinates, so every test is an exact integer comparison.
#include "sky_internal.h"

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
__global__ __launch_bounds__(SKY_WG) void k_ingest(const float *__restrict__ pts, uint32_t n, int d,
                                                  int need_range, float *__restrict__ score, int gf_on,
                                                  GridSpec gg, uint32_t *occ, uint32_t *ctrl, float *bnd)
{
    uint32_t err = 0;
    if (bnd) {
        // per-workgroup bounds of every coordinate: bnd[wg*32 + k] = min, [.. + 16 + k] = max
        __shared__ float s_b[4][32];
        const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int k = 0; k < d; ++k) {
            float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
            for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
                const float x = pts[(size_t)k * n + i];
                lo = fminf(lo, x);
                hi = fmaxf(hi, x);
            }
            for (int o = 32; o > 0; o >>= 1) {
                lo = fminf(lo, __shfl_xor(lo, o, 64));
                hi = fmaxf(hi, __shfl_xor(hi, o, 64));
            }
            if (lane == 0) { s_b[wv][k] = lo; s_b[wv][16 + k] = hi; }
        }
        __syncthreads();
        if (threadIdx.x < (uint32_t)d) {
            const int k = threadIdx.x;
            bnd[blockIdx.x * 32 + k] = fminf(fminf(s_b[0][k], s_b[1][k]), fminf(s_b[2][k], s_b[3][k]));
            bnd[blockIdx.x * 32 + 16 + k] =
                fmaxf(fmaxf(s_b[0][16 + k], s_b[1][16 + k]), fmaxf(s_b[2][16 + k], s_b[3][16 + k]));
        }
    }
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        float s = 0.0f;
        uint32_t cell = 0, mult = 1;
        for (int k = 0; k < d; ++k) {
            const float x = pts[(size_t)k * n + i];
            const uint32_t u = __float_as_uint(x);
            if ((u & 0x7f800000u) == 0x7f800000u) err |= 1u;
            else if (need_range && !(x >= 0.0f && x <= 1.0f)) err |= 2u;
            s = (k == 0) ? x : s + x;
            if (gf_on) {
                cell += grid_digit(x, gg.m[k]) * mult;
                mult *= (uint32_t)gg.m[k];
            }
        }
        if (score) score[i] = s;
        if (gf_on) {
            const uint32_t bit = 1u << (cell & 31);
            if (!(occ[cell >> 5] & bit)) atomicOr(&occ[cell >> 5], bit);
        }
    }
    if (err) atomicOr(&ctrl[C_ERR], err);
}

static uint32_t ingest_blocks(uint32_t n)
{
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    return blocks > SKY_INGEST_MAX_WG ? SKY_INGEST_MAX_WG : blocks;
}

hipError_t launch_ingest(const float *pts, uint32_t n, int d, int need_range, float *score, int gf_on,
                         const GridSpec &gg, uint32_t *occ, uint32_t *ctrl, float *bnd, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ingest, dim3(ingest_blocks(n)), dim3(SKY_WG), 0, s, pts, n, d, need_range, score, gf_on,
                       gg, occ, ctrl, bnd);
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

// One wave per quantised coordinate: reduce the per-workgroup bounds.
__global__ __launch_bounds__(1024) void k_zorder_scale(const float *__restrict__ bnd, uint32_t nblk, int b,
                                                      float *zq)
{
    const uint32_t lane = threadIdx.x & 63, k = threadIdx.x >> 6;
    float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
    for (uint32_t i = lane; i < nblk; i += 64) {
        lo = fminf(lo, bnd[i * 32 + k]);
        hi = fmaxf(hi, bnd[i * 32 + 16 + k]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    const float r = hi - lo;
    float sc = (r > 0.0f && r < __builtin_huge_valf()) ? (float)(1u << b) / r : 0.0f;
    if (!(sc < __builtin_huge_valf())) sc = 0.0f;
    if (lane == 0) {
        zq[k] = lo;
        zq[16 + k] = sc;
    }
}

hipError_t launch_zorder_scale(const float *bnd, uint32_t n, int d, int zbits, float *zq, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int b, nz;
    zorder_layout(d, zbits > 32 ? 32 : zbits, &b, &nz);
    hipLaunchKernelGGL(k_zorder_scale, dim3(1), dim3(64 * nz), 0, s, bnd, ingest_blocks(n), b, zq);
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

// ------------------------------------------------------------------ top-k select
// The k smallest points by (score, id) -- Sorted representatives take the
// coordinate sum, learned ones the MLP score (Section 4.1). MSB-first radix
// select over the unique 64-bit key (map(score) << 32 | id), 8 bits per pass.
__device__ __forceinline__ uint64_t sel_key(const float *score, uint32_t i)
{
    return ((uint64_t)ordmap(score[i]) << 32) | i;
}

__global__ __launch_bounds__(SKY_WG) void k_sel_hist(const float *__restrict__ score, uint32_t n,
                                                    const uint32_t *ctrl, uint32_t *hist, int shift)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = ((uint64_t)ctrl[C_SEL_PHI] << 32) | ctrl[C_SEL_PLO];
    const int hs = shift + 8;
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        const uint64_t key = sel_key(score, i);
        if (hs >= 64 || (key >> hs) == (prefix >> hs)) atomicAdd(&h[(uint32_t)(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(SKY_WG) void k_sel_pick(uint32_t *ctrl, uint32_t *hist, int shift)
{
    __shared__ uint32_t s[256];
    const uint32_t t = threadIdx.x;
    const uint32_t v = hist[t];
    s[t] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t y = t >= (uint32_t)o ? s[t - o] : 0;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    const uint32_t incl = s[t], excl = incl - v;
    const uint32_t k = ctrl[C_SEL_K];
    __syncthreads();
    if (v && excl < k && k <= incl) {
        uint64_t prefix = ((uint64_t)ctrl[C_SEL_PHI] << 32) | ctrl[C_SEL_PLO];
        prefix |= (uint64_t)t << shift;
        ctrl[C_SEL_PLO] = (uint32_t)prefix;
        ctrl[C_SEL_PHI] = (uint32_t)(prefix >> 32);
        ctrl[C_SEL_K] = k - excl;
    }
    hist[t] = 0;
}

__global__ __launch_bounds__(SKY_WG) void k_sel_collect(const float *__restrict__ score, uint32_t n,
                                                       uint32_t *ctrl, uint64_t *cand)
{
    const uint64_t thr = ((uint64_t)ctrl[C_SEL_PHI] << 32) | ctrl[C_SEL_PLO];
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        const uint64_t key = sel_key(score, i);
        if (key <= thr) {
            const uint32_t slot = atomicAdd(&ctrl[C_NCAND], 1u);
            if (slot < SKY_MAXREPS) cand[slot] = key;
        }
    }
}

hipError_t launch_topk(const float *score, uint32_t n, int k, uint32_t *ctrl, uint32_t *hist256,
                       uint64_t *cand, hipStream_t s)
{
    if (n == 0 || k <= 0) return hipSuccess;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 2048) blocks = 2048;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist, dim3(blocks), dim3(SKY_WG), 0, s, score, n, ctrl, hist256, shift);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(SKY_WG), 0, s, ctrl, hist256, shift);
    }
    hipLaunchKernelGGL(k_sel_collect, dim3(blocks), dim3(SKY_WG), 0, s, score, n, ctrl, cand);
    return hipGetLastError();
}

// Sort the (at most 256) candidates, build their records and apply the
// representative self-filter: a representative dominated by another one is
// discarded before the set is shared (Section 4.1). Kept records are
// compacted in score order into krec.
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_reps_finalize(const float *__restrict__ pts, uint32_t n, int d,
                                                         const uint64_t *__restrict__ cand, uint32_t *ctrl,
                                                         uint32_t *rep_ids, uint8_t *rep_keep, uint32_t *krec)
{
    __shared__ uint64_t sk[SKY_MAXREPS];
    __shared__ uint32_t rec[SKY_MAXREPS * DP];
    __shared__ uint32_t s_tmp[4];
    const uint32_t t = threadIdx.x;
    uint32_t c = ctrl[C_NCAND];
    if (c > SKY_MAXREPS) c = SKY_MAXREPS;
    sk[t] = t < c ? cand[t] : ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= SKY_MAXREPS; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            const uint32_t partner = t ^ stride;
            if (partner > t) {
                const bool up = (t & size) == 0;
                const uint64_t a = sk[t], b = sk[partner];
                if ((a > b) == up) { sk[t] = b; sk[partner] = a; }
            }
            __syncthreads();
        }
    }
    const uint32_t id = (uint32_t)sk[t];
    if (t < c) {
        uint64_t K = 0;
        for (int k = 0; k < DP - 2; ++k) {
            const uint32_t w = (k < d) ? ordmap(pts[(size_t)k * n + id]) : 0u;
            rec[t * DP + k] = w;
            K += w;
        }
        rec[t * DP + DP - 2] = (uint32_t)K;
        rec[t * DP + DP - 1] = (uint32_t)(K >> 32);
    }
    __syncthreads();
    bool keep = t < c;
    if (keep) {
        const uint64_t Kt = ((uint64_t)rec[t * DP + DP - 1] << 32) | rec[t * DP + DP - 2];
        for (uint32_t j = 0; j < c && keep; ++j) {
            if (j == t) continue;
            bool dm = true;
            for (int k = 0; k < DP - 2; ++k) dm &= rec[j * DP + k] <= rec[t * DP + k];
            const uint64_t Kj = ((uint64_t)rec[j * DP + DP - 1] << 32) | rec[j * DP + DP - 2];
            if (dm && Kj != Kt) keep = false;
        }
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

hipError_t launch_reps_finalize(const float *pts, uint32_t n, int d, const uint64_t *cand, uint32_t *ctrl,
                                uint32_t *rep_ids, uint8_t *rep_keep, uint32_t *krec, hipStream_t s)
{
    const int DP = sky_dp(d);
#define R_CASE(X)                                                                                     \
    case X:                                                                                           \
        hipLaunchKernelGGL(k_reps_finalize<X>, dim3(1), dim3(SKY_WG), 0, s, pts, n, d, cand, ctrl, rep_ids, \
                           rep_keep, krec);                                                           \
        break;
    switch (DP) {
        R_CASE(4) R_CASE(8) R_CASE(12) R_CASE(16) R_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef R_CASE
    return hipGetLastError();
}

__global__ void k_fill_zero_tail(uint32_t *p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
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
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_filter(const float *__restrict__ pts, uint32_t n, int d,
                                                  int gf_on, GridSpec gg, const uint32_t *__restrict__ gdom,
                                                  int use_reps, const uint32_t *__restrict__ krec,
                                                  int part_kind, GridSpec pg, AngSpec ag,
                                                  uint32_t *__restrict__ part, uint32_t *part_hist, int np,
                                                  uint8_t *__restrict__ alive, uint32_t *ctrl, uint32_t *grid_cnt)
{
    constexpr int ND = DP - 2;
    __shared__ uint32_t s_hist[4096];
    const uint32_t nk = use_reps ? __builtin_amdgcn_readfirstlane(ctrl[C_NREPS_KEPT]) : 0u;
    const bool lds_hist = part_kind != P_NONE && part_kind != P_SLICED && np <= 4096;
    if (lds_hist)
        for (int i = threadIdx.x; i < np; i += SKY_WG) s_hist[i] = 0;
    __syncthreads();
    uint32_t cnt_grid = 0, cnt_surv = 0;
    for (uint32_t base = blockIdx.x * SKY_WG; base < n; base += gridDim.x * SKY_WG) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < n;
        const uint32_t ii = valid ? i : n - 1;
        float x[ND];
        uint32_t w[ND];
        uint64_t K = 0;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            x[k] = k < d ? pts[(size_t)k * n + ii] : 0.0f;
            w[k] = (k < d) ? ordmap(x[k]) : 0u;
            K += w[k];
        }
        bool a = valid;
        if (gf_on && valid) {
            uint32_t cell = 0, mult = 1;
            for (int k = 0; k < d; ++k) {
                cell += grid_digit(x[k], gg.m[k]) * mult;
                mult *= (uint32_t)gg.m[k];
            }
            if ((gdom[cell >> 5] >> (cell & 31)) & 1u) a = false;
        }
        cnt_grid += a ? 1u : 0u;
        // representatives: read-only, wave-uniform records -> scalar loads, scalar operands
        // four records per batch: their scalar loads are issued together
        for (uint32_t r = 0; r < nk; r += 4) {
            if ((r & 15) == 0 && !__any(a)) break;
            uint32_t rr[4][DP];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < DP; ++k) rr[q][k] = krec[(r + q) * DP + k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t Kr = ((uint64_t)rr[q][DP - 1] << 32) | rr[q][DP - 2];
                bool dm = Kr != K;
#pragma unroll
                for (int k = 0; k < ND; ++k) dm = dm & (rr[q][k] <= w[k]);
                a = a & !dm;
            }
        }
        cnt_surv += a ? 1u : 0u;
        if (valid) {
            uint32_t pid = 0;
            if (part_kind == P_GRID) {
                uint32_t mult = 1;
                for (int k = 0; k < d; ++k) {
                    pid += grid_digit(x[k], pg.m[k]) * mult;
                    mult *= (uint32_t)pg.m[k];
                }
            } else if (part_kind == P_ANGULAR) {
                uint32_t mult = 1;
                for (int a2 = 0; a2 < d - 1; ++a2) {
                    double S = 0.0;
                    for (int j = a2 + 1; j < d; ++j) {
                        const double xj = (double)x[j];
                        S = __dadd_rn(S, __dmul_rn(xj, xj));
                    }
                    const double xi = (double)x[a2];
                    const double x2 = __dmul_rn(xi, xi);
                    uint32_t digit = 0;
                    for (int k = 1; k < ag.m[a2]; ++k)
                        if (S >= __dmul_rn(x2, ag.T[a2][k])) digit = (uint32_t)k;
                    pid += digit * mult;
                    mult *= (uint32_t)ag.m[a2];
                }
            }
            if (part_kind == P_GRID || part_kind == P_ANGULAR) {
                part[i] = pid;
                if (lds_hist) atomicAdd(&s_hist[pid], 1u);
                else atomicAdd(&part_hist[pid], 1u);
            }
            alive[i] = a ? 1 : 0;
        }
    }
    // per-workgroup count of grid survivors (summed later; a global atomic per
    // wave on one address would serialise). The survivor count itself is
    // produced by the compaction that follows.
    (void)cnt_surv;
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
                         const GridSpec &pg, const AngSpec &ag, uint32_t *part, uint32_t *part_hist, int np,
                         uint8_t *alive, uint32_t *ctrl, uint32_t *grid_cnt, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero_tail, dim3(1), dim3(SKY_WG), 0, s, grid_cnt, blocks);
    const int DP = sky_dp(d);
#define F_CASE(X)                                                                                           \
    case X:                                                                                                 \
        hipLaunchKernelGGL(k_filter<X>, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, d, gf_on, gg, gdom,      \
                           use_reps, krec, part_kind, pg, ag, part, part_hist, np, alive, ctrl, grid_cnt); \
        break;
    switch (DP) {
        F_CASE(4) F_CASE(8) F_CASE(12) F_CASE(16) F_CASE(20)
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
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 4096) blocks = 4096;
    if (n == 0) blocks = 0;
    hipLaunchKernelGGL(k_sum_grid, dim3(1), dim3(SKY_WG), 0, s, grid_cnt, blocks, ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Sliced partitioning
// Rank of every point in the order (x_s, then the other coordinates, then id),
// a total order and a linear extension of dominance; rank r goes to slice
// floor(r p / N) (Section 3.4). The ranks come from a stable LSD sort: first by
// x_s alone (ties then stay in id order); if a run of equal x_s straddles a
// slice boundary the host re-sorts lexicographically, coordinate by coordinate
// from the least significant one.
__global__ __launch_bounds__(SKY_WG) void k_sliced_init(const float *__restrict__ pts, uint32_t n, int coord,
                                                       uint64_t *keys, uint32_t *vals, int rekey_only)
{
    for (uint32_t i = blockIdx.x * SKY_WG + threadIdx.x; i < n; i += gridDim.x * SKY_WG) {
        uint32_t id = i;
        if (rekey_only) id = vals[i];
        else vals[i] = i;
        keys[i] = ordmap(pts[(size_t)coord * n + id]);
    }
}

hipError_t launch_sliced_init(const float *pts, uint32_t n, int coord, uint64_t *keys, uint32_t *vals,
                              int rekey_only, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_sliced_init, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, coord, keys, vals, rekey_only);
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

// ------------------------------------------------------------------ chunk table
// Partition j's points [poff[j], poff[j+1]) are cut into query groups of B
// points; nch[j] = their number and st_off the exclusive scan (group c of
// partition j is number st_off[j] + c). ctrl[which] = total groups, ctrl[C_MAXC]
// = the largest nch. One workgroup: thread t owns a contiguous range of
// partitions, so a single block scan suffices.
__global__ __launch_bounds__(1024) void k_chunk_table(const uint32_t *__restrict__ poff, int np, int B,
                                                      uint32_t *nch, uint32_t *st_off, uint32_t *ctrl, int which)
{
    __shared__ uint32_t s_w[16], s_m[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t per = ((uint32_t)np + 1023) / 1024;
    const uint32_t j0 = min((uint32_t)np, t * per), j1 = min((uint32_t)np, j0 + per);
    uint32_t sum = 0, mx = 0;
    for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t c = (poff[j + 1] - poff[j] + B - 1) / B;
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
        const uint32_t c = (poff[j + 1] - poff[j] + B - 1) / B;
        nch[j] = c;
        st_off[j] = run;
        run += c;
    }
    if (t == 0) {
        st_off[np] = tot;
        ctrl[which] = tot;
        ctrl[C_MAXC] = M;
    }
}

// gpart[g] = the partition of query group g (largest j with st_off[j] <= g).
__global__ __launch_bounds__(SKY_WG) void k_group_part(const uint32_t *__restrict__ st_off, int np,
                                                      const uint32_t *ctrl, int which, uint32_t *gpart)
{
    const uint32_t G = ctrl[which];
    for (uint32_t g = blockIdx.x * SKY_WG + threadIdx.x; g < G; g += gridDim.x * SKY_WG) {
        int lo = 0, hi = np - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (st_off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        gpart[g] = (uint32_t)lo;
    }
}

hipError_t launch_chunk_table(const uint32_t *poff, int np, int B, uint32_t *nch, uint32_t *st_off, uint32_t *gpart,
                              uint32_t *ctrl, int which, uint32_t g_max, hipStream_t s)
{
    hipLaunchKernelGGL(k_chunk_table, dim3(1), dim3(1024), 0, s, poff, np, B, nch, st_off, ctrl, which);
    uint32_t blocks = (g_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_group_part, dim3(blocks), dim3(SKY_WG), 0, s, st_off, np, ctrl, which, gpart);
    return hipGetLastError();
}
