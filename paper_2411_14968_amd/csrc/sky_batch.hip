// Kernels of the batched skyline: many independent instances in one launch
// sequence. The instance is an outer partition level of Algorithm 2: instance
// i's points are a contiguous range of a group array, its Sliced partitions
// are the global partitions i*p .. i*p+p-1, its representatives prune only its
// own points (Section 4.1), and the NoSeq merge (Proposition 2) looks only at
// earlier slices of the same instance. Instances of one group share a record
// width; an instance with fewer coordinates than the group gets zero
// coordinates, equal for all its points, which changes no dominance relation.
//
// Per group: goff[i] (group point offset of instance i, goff[ng] = NT), foff[i]
// (float offset of instance i in the caller's packed input, which holds each
// instance as SoA (d_i, N_i)), gd[i] = d_i.
#include "sky_internal.h"
#include "sky_domtest.h"

__device__ __forceinline__ uint64_t lane_below_mask()
{
    const uint32_t lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint32_t batch_inst(const uint32_t *__restrict__ goff, int ng, uint32_t gi)
{
    int lo = 0, hi = ng - 1;   // largest i with goff[i] <= gi
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (goff[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    return (uint32_t)lo;
}

// Group SoA (dg, NT) from the packed instances, and the instance of every point.
__global__ __launch_bounds__(SKY_WG) void k_batch_pack(const float *__restrict__ pts, const int64_t *__restrict__ foff,
                                                      const uint32_t *__restrict__ goff,
                                                      const int32_t *__restrict__ gd, int ng, uint32_t NT, int dg,
                                                      float *__restrict__ out, uint32_t *__restrict__ inst)
{
    for (uint32_t gi = blockIdx.x * SKY_WG + threadIdx.x; gi < NT; gi += gridDim.x * SKY_WG) {
        const uint32_t i = batch_inst(goff, ng, gi);
        const uint32_t li = gi - goff[i], ni = goff[i + 1] - goff[i];
        const int di = gd[i];
        const float *src = pts + foff[i];
        for (int k = 0; k < dg; ++k) out[(size_t)k * NT + gi] = k < di ? src[(size_t)k * ni + li] : 0.0f;
        inst[gi] = i;
    }
}

// keys = (instance, map(v)), vals = group index: sorted, each instance's points
// form one run in ascending v (ties in index order).
__global__ __launch_bounds__(SKY_WG) void k_batch_keys(const uint32_t *__restrict__ inst,
                                                      const float *__restrict__ v, uint32_t NT, uint64_t *keys,
                                                      uint32_t *vals)
{
    for (uint32_t gi = blockIdx.x * SKY_WG + threadIdx.x; gi < NT; gi += gridDim.x * SKY_WG) {
        keys[gi] = ((uint64_t)inst[gi] << 32) | ordmap(v[gi]);
        vals[gi] = gi;
    }
}

// Sorted representatives of instance i = blockIdx.x: its first c = min(nreps,
// N_i) points in (sum, index) order; the self-filter drops one dominated by
// another; kept records go to krec[i] in that order, padded to a multiple of 4
// with all-ones records (no finite point is dominated by one); nk[i] = kept.
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_batch_reps(const float *__restrict__ pts, uint32_t NT, int d,
                                                      const uint32_t *__restrict__ vals,
                                                      const uint32_t *__restrict__ goff, int nreps,
                                                      uint32_t *krec, uint32_t *nk)
{
    __shared__ uint32_t rec[SKY_MAXREPS * DP];
    __shared__ uint32_t s_tmp[4];
    const uint32_t i = blockIdx.x, t = threadIdx.x;
    const uint32_t ni = goff[i + 1] - goff[i];
    const uint32_t c = min((uint32_t)nreps, ni);
    if (t < c) {
        const uint32_t id = vals[goff[i] + t];
        uint64_t K = 0;
        for (int k = 0; k < DP - 2; ++k) {
            const uint32_t w = (k < d) ? ordmap(pts[(size_t)k * NT + id]) : 0u;
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
    const int lane = t & 63, wv = t >> 6;
    const uint64_t m = __ballot(keep);
    if (lane == 0) s_tmp[wv] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t r = (uint32_t)__popcll(m & lane_below_mask());
    for (int w = 0; w < wv; ++w) r += s_tmp[w];
    const uint32_t tot = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    uint32_t *kr = krec + (size_t)i * SKY_MAXREPS * DP;
    if (keep)
        for (int k = 0; k < DP; ++k) kr[r * DP + k] = rec[t * DP + k];
    if (t >= tot && t < ((tot + 3u) & ~3u))
        for (int k = 0; k < DP; ++k) kr[t * DP + k] = 0xFFFFFFFFu;
    if (t == 0) nk[i] = tot;
}

// Representative Filtering inside each instance: alive[gi] = 0 if a kept
// representative of gi's instance dominates it (Def. 1 on the mapped images).
// A lane takes FPP points, rows of live masks. When every point of the wave
// belongs to one instance (instances are contiguous, so nearly every wave),
// the representatives are wave-uniform: read through scalar loads, four per
// batch, and tested with the exec-mask chains, stopping early once every row
// is empty. A wave that spans instances tests each lane's own set.
template <int DP, int NC>
__global__ __launch_bounds__(SKY_WG) void k_batch_filter(const float *__restrict__ pts, uint32_t NT, int d,
                                                        const uint32_t *__restrict__ inst,
                                                        const uint32_t *__restrict__ krec,
                                                        const uint32_t *__restrict__ nk, uint8_t *__restrict__ alive)
{
    constexpr int ND = DP - 2, FPP = DP <= 16 ? 2 : 1;
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t base = blockIdx.x * SKY_WG * FPP; base < NT; base += gridDim.x * SKY_WG * FPP) {
        uint32_t w[FPP][ND], ins[FPP];
        uint64_t K[FPP];
        bool a[FPP];
#pragma unroll
        for (int q = 0; q < FPP; ++q) {
            const uint32_t gi = base + q * SKY_WG + threadIdx.x;
            const uint32_t gc = gi < NT ? gi : NT - 1;
            K[q] = 0;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                const float x = pts[(size_t)(k < d ? k : d - 1) * NT + gc];
                w[q][k] = k < d ? ordmap(x) : 0u;
                K[q] += w[q][k];
            }
            ins[q] = inst[gc];
            a[q] = gi < NT;
        }
        const uint32_t i0 = __builtin_amdgcn_readfirstlane(ins[0]);
        bool same = true;
#pragma unroll
        for (int q = 0; q < FPP; ++q) same = same && ins[q] == i0;
        if (__ballot(!same) == 0) {   // wave-uniform: one instance
            const uint32_t nr = (__builtin_amdgcn_readfirstlane(nk[i0]) + 3u) & ~3u;
            const uint32_t *rp = krec + (size_t)i0 * SKY_MAXREPS * DP;
            uint64_t am[FPP];
#pragma unroll
            for (int q = 0; q < FPP; ++q) am[q] = __ballot(a[q]);
            for (uint32_t r = 0; r < nr; r += 4, rp += 4 * DP) {
                uint64_t any = 0;
#pragma unroll
                for (int q = 0; q < FPP; ++q) any |= am[q];
                if ((r & 15) == 0 && !any) break;
                uint32_t rr[4][DP];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int k = 0; k < DP; ++k) rr[u][k] = rp[u * DP + k];
#pragma unroll
                for (int u = 0; u < 4; ++u) test_rec<DP, NC, FPP>(rr[u], w, K, am);
            }
#pragma unroll
            for (int q = 0; q < FPP; ++q) a[q] = (am[q] >> lane) & 1ull;
        } else {
#pragma unroll
            for (int q = 0; q < FPP; ++q) {
                const uint32_t nr = (nk[ins[q]] + 3u) & ~3u;
                const uint32_t *kr = krec + (size_t)ins[q] * SKY_MAXREPS * DP;
                for (uint32_t r = 0; r < nr && a[q]; ++r) {
                    const uint32_t *rr = kr + (size_t)r * DP;
                    const uint64_t Kr = ((uint64_t)rr[DP - 1] << 32) | rr[DP - 2];
                    bool dm = Kr != K[q];
#pragma unroll
                    for (int k = 0; k < ND; ++k) dm = dm & (rr[k] <= w[q][k]);
                    a[q] = a[q] & !dm;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < FPP; ++q) {
            const uint32_t gi = base + q * SKY_WG + threadIdx.x;
            if (gi < NT) alive[gi] = a[q] ? 1 : 0;
        }
    }
}

// Equal x_s values on both sides of a slice boundary of some instance.
__global__ __launch_bounds__(SKY_WG) void k_batch_sliced_check(const uint64_t *__restrict__ keys,
                                                              const uint32_t *__restrict__ goff, int ng, int p,
                                                              uint32_t *ctrl)
{
    const uint32_t nb = (uint32_t)ng * (uint32_t)(p - 1);
    for (uint32_t q = blockIdx.x * SKY_WG + threadIdx.x; q < nb; q += gridDim.x * SKY_WG) {
        const uint32_t i = q / (uint32_t)(p - 1), j = q % (uint32_t)(p - 1) + 1;
        const uint32_t ni = goff[i + 1] - goff[i];
        const uint64_t r = ((uint64_t)j * ni + p - 1) / p;   // first rank of slice j
        if (r >= 1 && r < ni && keys[goff[i] + r - 1] == keys[goff[i] + r]) atomicOr(&ctrl[C_TIE], 1u);
    }
}

// Sorted position -> global partition: instance i's rank r goes to slice
// floor(r * p / N_i), partition i * p + slice.
__global__ __launch_bounds__(SKY_WG) void k_batch_sliced_assign(const uint32_t *__restrict__ vals,
                                                               const uint32_t *__restrict__ inst,
                                                               const uint32_t *__restrict__ goff, uint32_t NT, int p,
                                                               uint32_t *__restrict__ part)
{
    for (uint32_t pos = blockIdx.x * SKY_WG + threadIdx.x; pos < NT; pos += gridDim.x * SKY_WG) {
        const uint32_t gi = vals[pos];
        const uint32_t i = inst[gi];
        const uint32_t r = pos - goff[i], ni = goff[i + 1] - goff[i];
        part[gi] = i * (uint32_t)p + (uint32_t)(((uint64_t)r * (uint32_t)p) / ni);
    }
}

// Skyline points of each instance: popcount of its range of the bitmap.
__global__ __launch_bounds__(SKY_WG) void k_batch_counts(const uint32_t *__restrict__ bits,
                                                        const uint32_t *__restrict__ goff, uint32_t *cnt)
{
    __shared__ uint32_t s_tmp[4];
    const uint32_t i = blockIdx.x;
    const uint32_t b0 = goff[i], b1 = goff[i + 1];
    uint32_t c = 0;
    for (uint32_t w = (b0 >> 5) + threadIdx.x; w <= (b1 == 0 ? 0 : (b1 - 1) >> 5) && b1 > b0; w += SKY_WG) {
        uint32_t m = bits[w];
        const uint32_t lo = w << 5;
        if (lo < b0) m &= ~0u << (b0 - lo);
        if (lo + 32 > b1) m &= (b1 - lo >= 32) ? ~0u : ((1u << (b1 - lo)) - 1u);
        c += __popc(m);
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[i] = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
}

static uint32_t grid_for(uint32_t n)
{
    uint32_t b = (n + SKY_WG - 1) / SKY_WG;
    if (b < 1) b = 1;
    return b > 8192 ? 8192 : b;
}

hipError_t launch_batch_pack(const float *pts, const int64_t *foff, const uint32_t *goff, const int32_t *gd, int ng,
                             uint32_t NT, int dg, float *out, uint32_t *inst, hipStream_t s)
{
    if (NT == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_pack, dim3(grid_for(NT)), dim3(SKY_WG), 0, s, pts, foff, goff, gd, ng, NT, dg, out,
                       inst);
    return hipGetLastError();
}

hipError_t launch_batch_keys(const uint32_t *inst, const float *v, uint32_t NT, uint64_t *keys, uint32_t *vals,
                             hipStream_t s)
{
    if (NT == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_keys, dim3(grid_for(NT)), dim3(SKY_WG), 0, s, inst, v, NT, keys, vals);
    return hipGetLastError();
}

hipError_t launch_batch_reps(const float *pts, uint32_t NT, int d, const uint32_t *vals, const uint32_t *goff,
                             int ng, int nreps, uint32_t *krec, uint32_t *nk, hipStream_t s)
{
    if (ng == 0) return hipSuccess;
    const int DP = sky_dp(d);
#define BR_CASE(X)                                                                                          \
    case X:                                                                                                 \
        hipLaunchKernelGGL(k_batch_reps<X>, dim3(ng), dim3(SKY_WG), 0, s, pts, NT, d, vals, goff, nreps, krec, \
                           nk);                                                                             \
        break;
    switch (DP) {
        BR_CASE(4) BR_CASE(8) BR_CASE(12) BR_CASE(16) BR_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef BR_CASE
    return hipGetLastError();
}

hipError_t launch_batch_filter(const float *pts, uint32_t NT, int d, const uint32_t *inst, const uint32_t *krec,
                               const uint32_t *nk, uint8_t *alive, hipStream_t s)
{
    if (NT == 0) return hipSuccess;
    const int DP = sky_dp(d), NC = sky_nc(d);
    uint32_t blocks = (NT + 2 * SKY_WG - 1) / (2 * SKY_WG);
    if (blocks > 4096) blocks = 4096;
#define BF_CASE(X, C)                                                                                           \
    case X * 32 + C:                                                                                            \
        hipLaunchKernelGGL((k_batch_filter<X, C>), dim3(blocks), dim3(SKY_WG), 0, s, pts, NT, d, inst, krec, nk, \
                           alive);                                                                              \
        break;
    switch (DP * 32 + NC) {
        BF_CASE(4, 2) BF_CASE(8, 4) BF_CASE(8, 6) BF_CASE(12, 8) BF_CASE(12, 10) BF_CASE(16, 12) BF_CASE(16, 14)
        BF_CASE(20, 16)
        default: return hipErrorInvalidValue;
    }
#undef BF_CASE
    return hipGetLastError();
}

hipError_t launch_batch_sliced_check(const uint64_t *keys, const uint32_t *goff, int ng, int p, uint32_t *ctrl,
                                     hipStream_t s)
{
    if (ng == 0 || p < 2) return hipSuccess;
    hipLaunchKernelGGL(k_batch_sliced_check, dim3(grid_for((uint32_t)ng * (uint32_t)(p - 1))), dim3(SKY_WG), 0, s,
                       keys, goff, ng, p, ctrl);
    return hipGetLastError();
}

hipError_t launch_batch_sliced_assign(const uint32_t *vals, const uint32_t *inst, const uint32_t *goff, uint32_t NT,
                                      int p, uint32_t *part, hipStream_t s)
{
    if (NT == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_sliced_assign, dim3(grid_for(NT)), dim3(SKY_WG), 0, s, vals, inst, goff, NT, p, part);
    return hipGetLastError();
}

hipError_t launch_batch_counts(const uint32_t *bits, const uint32_t *goff, int ng, uint32_t *cnt, hipStream_t s)
{
    if (ng == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_counts, dim3(ng), dim3(SKY_WG), 0, s, bits, goff, cnt);
    return hipGetLastError();
}
