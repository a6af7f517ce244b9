// The dominance-test kernels: local skylines with SFS semantics (Algorithm 1
// inside each partition of Algorithm 2) and the NoSeq merge (Proposition 2).
//
// Records (see sky_internal.h) hold order-preserving uint32 images of the
// coordinates plus K = their sum; w dominates t iff all coordinate words of w
// are <= those of t and K(w) != K(t). Inside a partition the points are sorted
// by a key that is a linear extension of dominance, so a point can only be
// dominated by points earlier in the order (the topological-sort property of
// Section 2 that SFS relies on).
#include "sky_internal.h"

__device__ __forceinline__ uint64_t rec_key(const uint32_t *r, int DP)
{
    return ((uint64_t)r[DP - 1] << 32) | r[DP - 2];
}

// Test one staged record (LDS, uniform across the wave) against the lane's
// PPL points; clears al[q] for dominated points.
template <int DP, int PPL>
__device__ __forceinline__ void test_rec(const uint32_t *__restrict__ r, const uint32_t (&x)[PPL][DP - 2],
                                         const uint64_t (&K)[PPL], bool (&al)[PPL])
{
    uint32_t w[DP];
#pragma unroll
    for (int k = 0; k < DP / 4; ++k) {
        const uint4 v = reinterpret_cast<const uint4 *>(r)[k];
        w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
    }
    const uint64_t Kw = ((uint64_t)w[DP - 1] << 32) | w[DP - 2];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        bool dm = Kw != K[q];
#pragma unroll
        for (int k = 0; k < DP - 2; ++k) dm &= w[k] <= x[q][k];
        al[q] = al[q] && !dm;
    }
}

template <int PPL>
__device__ __forceinline__ bool any_alive(const bool (&al)[PPL])
{
    bool a = false;
#pragma unroll
    for (int q = 0; q < PPL; ++q) a |= al[q];
    return a;
}

// Scan records src[0..cnt) (global, AoS) against the lane points: the wave
// stages 64 records at a time in its LDS tile and every lane tests them in
// order; the wave stops as soon as none of its points is alive.
template <int DP, int PPL>
__device__ __forceinline__ void scan_records(const uint32_t *src, uint32_t cnt, uint32_t *tile,
                                             const uint32_t (&x)[PPL][DP - 2], const uint64_t (&K)[PPL],
                                             bool (&al)[PPL])
{
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t w0 = 0; w0 < cnt; w0 += 64) {
        if (!__any(any_alive<PPL>(al))) return;
        const uint32_t nw = min(64u, cnt - w0);
        if (lane < nw) {
            const uint4 *s = reinterpret_cast<const uint4 *>(src + (size_t)(w0 + lane) * DP);
            uint4 *d = reinterpret_cast<uint4 *>(tile + lane * DP);
#pragma unroll
            for (int k = 0; k < DP / 4; ++k) d[k] = s[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t w = 0; w < nw; ++w) {
            if ((w & 7) == 0 && w && !__any(any_alive<PPL>(al))) break;
            test_rec<DP, PPL>(tile + w * DP, x, K, al);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Next work ticket of a persistent wave. All 64 lanes add 1 (the counter
// advances by 64 per ticket) so the call sits in no lane-divergent branch; the
// wave's ticket is lane 0's old value / 64. Waves work independently: these
// kernels have no workgroup barrier at all.
__device__ __forceinline__ uint32_t wave_ticket(uint32_t *counter)
{
    const uint32_t v = atomicAdd(counter, 1u);
    return __builtin_amdgcn_readfirstlane(v) >> 6;
}

template <int DP, int PPL>
__device__ __forceinline__ void load_points(const uint32_t *__restrict__ src, uint32_t len, uint32_t (&x)[PPL][DP - 2],
                                            uint64_t (&K)[PPL], bool (&al)[PPL])
{
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const uint32_t o = q * 64 + lane;
        al[q] = o < len;
        const uint4 *s = reinterpret_cast<const uint4 *>(src + (size_t)(al[q] ? o : 0) * DP);
        uint32_t w[DP];
#pragma unroll
        for (int k = 0; k < DP / 4; ++k) {
            const uint4 v = s[k];
            w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
        }
#pragma unroll
        for (int k = 0; k < DP - 2; ++k) x[q][k] = w[k];
        K[q] = ((uint64_t)w[DP - 1] << 32) | w[DP - 2];
    }
}

// ------------------------------------------------------------------ local skyline
// Persistent waves take chunks (64 * PPL consecutive points of one partition,
// lane l holds chunk offsets q * 64 + l) from a ticket counter. A point of
// chunk c is in the local skyline u_j iff no earlier point of the partition
// dominates it. It is tested
//  1. against each earlier chunk c' < c: the compacted local skyline of c' if
//     c' has been published, else all raw points of c' (testing against every
//     earlier point is exact too, since a dominated dominator is itself
//     dominated by an earlier skyline point) -- so no wave ever waits;
//  2. against the earlier points of its own chunk that survived step 1 (a
//     dominator killed in step 1 was killed by a point that also dominates).
// The chunk then publishes its skyline points, compacted in key order, with a
// release store of (count + 1) to its state word.
template <int DP, int PPL>
__global__ __launch_bounds__(256) void k_local_wave(const uint32_t *__restrict__ raw, uint32_t *win, uint32_t *wpos,
                                                   uint32_t *state, const uint32_t *__restrict__ poff,
                                                   const uint32_t *__restrict__ st_off,
                                                   const uint32_t *__restrict__ table, uint32_t *ctrl,
                                                   int ticket_slot, int nchunk_slot, uint8_t *in_u)
{
    constexpr int B = 64 * PPL, ND = DP - 2;
    __shared__ __attribute__((aligned(16))) uint32_t s_tile[4][64 * DP];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *tile = s_tile[wv];
    const uint32_t nchunks = __builtin_amdgcn_readfirstlane(ctrl[nchunk_slot]);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (;;) {
        const uint32_t g = wave_ticket(&ctrl[ticket_slot]);
        if (g >= nchunks) break;
        const uint32_t j = __builtin_amdgcn_readfirstlane(table[2 * g]);
        const uint32_t c = __builtin_amdgcn_readfirstlane(table[2 * g + 1]);
        const uint32_t pbeg = __builtin_amdgcn_readfirstlane(poff[j]);
        const uint32_t pend = __builtin_amdgcn_readfirstlane(poff[j + 1]);
        const uint32_t start = pbeg + c * B;
        const uint32_t len = min((uint32_t)B, pend - start);
        uint32_t x[PPL][ND];
        uint64_t K[PPL];
        bool al[PPL];
        load_points<DP, PPL>(raw + (size_t)start * DP, len, x, K, al);
        // 1. earlier chunks of the partition, strongest (smallest keys) first
        const uint32_t sbase = __builtin_amdgcn_readfirstlane(st_off[j]);
        for (uint32_t cp = 0; cp < c; ++cp) {
            if (!__any(any_alive<PPL>(al))) break;
            uint32_t st = __hip_atomic_load(&state[sbase + cp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st = __builtin_amdgcn_readfirstlane(st);
            const uint32_t cstart = pbeg + cp * B;
            if (st) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                scan_records<DP, PPL>(win + (size_t)cstart * DP, st - 1, tile, x, K, al);
            } else {
                scan_records<DP, PPL>(raw + (size_t)cstart * DP, (uint32_t)B, tile, x, K, al);
            }
        }
        // 2. earlier survivors of the own chunk (masks are wave-uniform)
        uint64_t m[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) m[q] = __ballot(al[q]);
#pragma unroll
        for (int q2 = 0; q2 < PPL; ++q2) {
            const uint32_t o0 = q2 * 64;
            if (o0 >= len || !__any(any_alive<PPL>(al))) break;
            const uint32_t nw = min(64u, len - o0);
            if (lane < nw) {
                const uint4 *s = reinterpret_cast<const uint4 *>(raw + (size_t)(start + o0 + lane) * DP);
                uint4 *d = reinterpret_cast<uint4 *>(tile + lane * DP);
#pragma unroll
                for (int k = 0; k < DP / 4; ++k) d[k] = s[k];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (uint32_t l2 = 0; l2 < nw; ++l2) {
                if (!((m[q2] >> l2) & 1ull)) continue;
                const uint32_t o2 = o0 + l2;
                bool keep[PPL];
#pragma unroll
                for (int q = 0; q < PPL; ++q) keep[q] = true;
                test_rec<DP, PPL>(tile + l2 * DP, x, K, keep);
#pragma unroll
                for (int q = 0; q < PPL; ++q)
                    if ((uint32_t)(q * 64) + lane > o2) al[q] = al[q] && keep[q];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // publish: flags, then the compacted records in key order
        uint32_t base = 0;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const uint32_t o = q * 64 + lane;
            if (o < len) in_u[start + o] = al[q] ? 1 : 0;
            const uint64_t mq = __ballot(al[q]);
            if (al[q]) {
                const uint32_t rank = base + (uint32_t)__popcll(mq & lt);
                uint32_t w[DP];
#pragma unroll
                for (int k = 0; k < ND; ++k) w[k] = x[q][k];
                w[DP - 2] = (uint32_t)K[q];
                w[DP - 1] = (uint32_t)(K[q] >> 32);
                uint4 *d = reinterpret_cast<uint4 *>(win + (size_t)(start + rank) * DP);
#pragma unroll
                for (int k = 0; k < DP / 4; ++k) d[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
                wpos[start + rank] = start + o;
            }
            base += (uint32_t)__popcll(mq);
        }
        __threadfence();
        __hip_atomic_store(&state[sbase + c], base + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int PPL>
static hipError_t local_wave_ppl(int DP, const uint32_t *raw, uint32_t *win, uint32_t *wpos, uint32_t *state,
                                 const uint32_t *poff, const uint32_t *st_off, const uint32_t *table, uint32_t *ctrl,
                                 int ticket_slot, int nchunk_slot, uint8_t *in_u, int n_wg, hipStream_t s)
{
#define L_CASE(X)                                                                                        \
    case X:                                                                                              \
        hipLaunchKernelGGL((k_local_wave<X, PPL>), dim3(n_wg), dim3(256), 0, s, raw, win, wpos, state, poff, \
                           st_off, table, ctrl, ticket_slot, nchunk_slot, in_u);                         \
        break;
    switch (DP) {
        L_CASE(4) L_CASE(8) L_CASE(12) L_CASE(16) L_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef L_CASE
    return hipGetLastError();
}

// Points per lane of the local-skyline kernel; a chunk is 64 * PPL points.
int local_sky_ppl(int d) { return sky_dp(d) <= 8 ? 2 : 1; }
int local_sky_chunk(int d) { return 64 * local_sky_ppl(d); }

hipError_t launch_local_sky(int d, const uint32_t *raw, uint32_t *win, uint32_t *wpos, uint32_t *state,
                            const uint32_t *poff, const uint32_t *st_off, const uint32_t *table, uint32_t *ctrl,
                            int ticket_slot, int nchunk_slot, uint8_t *in_u, int n_wg, hipStream_t s)
{
    const int DP = sky_dp(d);
    if (local_sky_ppl(d) == 2)
        return local_wave_ppl<2>(DP, raw, win, wpos, state, poff, st_off, table, ctrl, ticket_slot, nchunk_slot,
                                 in_u, n_wg, s);
    return local_wave_ppl<1>(DP, raw, win, wpos, state, poff, st_off, table, ctrl, ticket_slot, nchunk_slot, in_u,
                             n_wg, s);
}

// ------------------------------------------------------------------ union of local skylines
// Exclusive scan of the published chunk counts (partition-major), giving the
// dense position of every chunk's skyline records in u, the partition offsets
// upoff of u, |u| and the local skyline sizes.
__global__ __launch_bounds__(1024) void k_scan_states(const uint32_t *__restrict__ state,
                                                      const uint32_t *__restrict__ st_off, int np,
                                                      uint32_t *uoff_chunks, uint32_t *upoff, uint32_t *ctrl,
                                                      int nchunk_slot, int64_t *local_sizes)
{
    __shared__ uint32_t s[1024];
    const uint32_t cnt = ctrl[nchunk_slot];
    const uint32_t per = (cnt + 1023) / 1024;
    const uint32_t b = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t i = 0; i < per && b + i < cnt; ++i) sum += state[b + i] - 1u;
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - sum;
    for (uint32_t i = 0; i < per && b + i < cnt; ++i) {
        uoff_chunks[b + i] = run;
        run += state[b + i] - 1u;
    }
    uoff_chunks[cnt] = s[1023];   // written by every thread with the same value
    __syncthreads();
    for (int j = threadIdx.x; j <= np; j += 1024) upoff[j] = uoff_chunks[st_off[j]];
    if (threadIdx.x == 0) ctrl[C_NU] = s[1023];
    __syncthreads();
    if (local_sizes)
        for (int j = threadIdx.x; j < np; j += 1024) local_sizes[j] = (int64_t)(upoff[j + 1] - upoff[j]);
}

// Copy each chunk's published records into the dense u arrays (one workgroup
// per chunk, partition-major numbering).
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_compact_u(const uint32_t *__restrict__ win,
                                                     const uint32_t *__restrict__ wpos,
                                                     const uint32_t *__restrict__ state,
                                                     const uint32_t *__restrict__ poff,
                                                     const uint32_t *__restrict__ st_off, int np, int B,
                                                     const uint32_t *__restrict__ uoff_chunks,
                                                     const uint32_t *__restrict__ sid,
                                                     const uint64_t *__restrict__ skey, const uint32_t *ctrl,
                                                     int nchunk_slot, uint32_t *__restrict__ urec,
                                                     uint32_t *__restrict__ uid, uint64_t *__restrict__ ukey)
{
    const uint32_t nchunks = ctrl[nchunk_slot];
    for (uint32_t g = blockIdx.x; g < nchunks; g += gridDim.x) {
        // partition of chunk g: largest j with st_off[j] <= g (binary search)
        int lo = 0, hi = np - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (st_off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const uint32_t j = (uint32_t)lo;
        const uint32_t cstart = poff[j] + (g - st_off[j]) * (uint32_t)B;
        const uint32_t cnt = state[g] - 1u;
        const uint32_t dst = uoff_chunks[g];
        for (uint32_t e = threadIdx.x; e < cnt; e += SKY_WG) {
            const uint4 *s = reinterpret_cast<const uint4 *>(win + (size_t)(cstart + e) * DP);
            uint4 *d = reinterpret_cast<uint4 *>(urec + (size_t)(dst + e) * DP);
#pragma unroll
            for (int k = 0; k < DP / 4; ++k) d[k] = s[k];
            const uint32_t r = wpos[cstart + e];
            uid[dst + e] = sid[r];
            ukey[dst + e] = skey[r];
        }
    }
}

hipError_t launch_union(int d, const uint32_t *win, const uint32_t *wpos, const uint32_t *state,
                        const uint32_t *poff, const uint32_t *st_off, int np, int B, uint32_t *uoff_chunks,
                        uint32_t max_chunks, const uint32_t *sid, const uint64_t *skey, uint32_t *ctrl,
                        int nchunk_slot, uint32_t *urec, uint32_t *uid, uint64_t *ukey, uint32_t *upoff,
                        int64_t *local_sizes, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_states, dim3(1), dim3(1024), 0, s, state, st_off, np, uoff_chunks, upoff, ctrl,
                       nchunk_slot, local_sizes);
    uint32_t blocks = max_chunks < 1 ? 1 : max_chunks;
    if (blocks > 4096) blocks = 4096;
    const int DP = sky_dp(d);
#define U_CASE(X)                                                                                           \
    case X:                                                                                                 \
        hipLaunchKernelGGL(k_compact_u<X>, dim3(blocks), dim3(SKY_WG), 0, s, win, wpos, state, poff, st_off, \
                           np, B, uoff_chunks, sid, skey, ctrl, nchunk_slot, urec, uid, ukey);             \
        break;
    switch (DP) {
        U_CASE(4) U_CASE(8) U_CASE(12) U_CASE(16) U_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef U_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------ NoSeq merge
// Sky(r) = union_i Sky_{pd_i}(u_i) (Proposition 2): every point of u_i is
// tested against its partition's potential dominators pd_i, and survives iff
// none dominates it. pd_i: Sliced u_j, j < i; Grid u_j with c_j <= c_i in
// every dimension, j != i (the weak grid-dominance superset, always sound);
// Angular every u_j, j != i. Only points with a smaller (Q, K) key can
// dominate, and u_j is sorted by that key, so u_j is scanned up to the largest
// key of the query points.
// Work: tickets over (block of JB candidate partitions, query group of 64*PPL
// points of one u_i), the partition blocks outermost; for Sliced the blocks
// run from the nearest lower slice downwards. A query point killed by any
// ticket is marked dead, and later tickets of its group skip it.
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

template <int DP, int PPL>
__global__ __launch_bounds__(256) void k_merge_wave(const uint32_t *__restrict__ urec,
                                                   const uint64_t *__restrict__ ukey,
                                                   const uint32_t *__restrict__ upoff,
                                                   const uint32_t *__restrict__ table, int np, int JB,
                                                   int part_kind, GridSpec pg, uint32_t *ctrl, uint8_t *udead)
{
    constexpr int B = 64 * PPL, ND = DP - 2;
    __shared__ __attribute__((aligned(16))) uint32_t s_tile[4][64 * DP];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *tile = s_tile[wv];
    const uint32_t nq = __builtin_amdgcn_readfirstlane(ctrl[C_NCHUNK2]);
    const uint32_t JT = ((uint32_t)np + JB - 1) / JB;
    const uint64_t total = (uint64_t)nq * JT;
    for (;;) {
        const uint32_t t = wave_ticket(&ctrl[C_TICKET2]);
        if (t >= total) break;
        const uint32_t jt = t / nq, qg = t - jt * nq;
        const uint32_t i = __builtin_amdgcn_readfirstlane(table[2 * qg]);
        const uint32_t c = __builtin_amdgcn_readfirstlane(table[2 * qg + 1]);
        const uint32_t qstart = __builtin_amdgcn_readfirstlane(upoff[i]) + c * B;
        const uint32_t qlen = min((uint32_t)B, __builtin_amdgcn_readfirstlane(upoff[i + 1]) - qstart);
        uint32_t x[PPL][ND];
        uint64_t K[PPL];
        bool al[PPL], was[PPL];
        load_points<DP, PPL>(urec + (size_t)qstart * DP, qlen, x, K, al);
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            if (al[q] && udead[qstart + q * 64 + lane]) al[q] = false;
            was[q] = al[q];
        }
        if (!__any(any_alive<PPL>(al))) continue;
        // largest presort key among the group (points are key-sorted)
        const uint32_t last = min(qlen - 1, (uint32_t)((PPL - 1) * 64 + 63));
        const uint64_t kmax = ukey[qstart + last];
        for (int jj = 0; jj < JB; ++jj) {
            const uint32_t jidx = jt * JB + jj;
            if (jidx >= (uint32_t)np || !__any(any_alive<PPL>(al))) break;
            uint32_t j;
            bool pd;
            if (part_kind == P_SLICED) {
                pd = jidx < i;
                j = i - 1 - jidx;
            } else {
                j = jidx;
                pd = j != i && (part_kind != P_GRID || grid_weakly_below(j, i, pg));
            }
            if (!pd) continue;
            const uint32_t lo0 = __builtin_amdgcn_readfirstlane(upoff[j]);
            uint32_t lo = lo0, hi = __builtin_amdgcn_readfirstlane(upoff[j + 1]);
            while (lo < hi) {   // first position with key > kmax
                const uint32_t mid = (lo + hi) >> 1;
                if (ukey[mid] <= kmax) lo = mid + 1; else hi = mid;
            }
            lo = __builtin_amdgcn_readfirstlane(lo);
            scan_records<DP, PPL>(urec + (size_t)lo0 * DP, lo - lo0, tile, x, K, al);
        }
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            if (was[q] && !al[q]) udead[qstart + q * 64 + lane] = 1;
    }
}

__global__ __launch_bounds__(SKY_WG) void k_merge_finish(const uint8_t *__restrict__ udead,
                                                        const uint32_t *__restrict__ uid, const uint32_t *ctrl,
                                                        uint32_t *skybits)
{
    const uint32_t n = ctrl[C_NU];
    for (uint32_t r = blockIdx.x * SKY_WG + threadIdx.x; r < n; r += gridDim.x * SKY_WG)
        if (!udead[r]) {
            const uint32_t id = uid[r];
            atomicOr(&skybits[id >> 5], 1u << (id & 31));
        }
}

int merge_ppl(int d) { return sky_dp(d) <= 8 ? 4 : 2; }
int merge_chunk(int d) { return 64 * merge_ppl(d); }

hipError_t launch_merge_noseq(int d, const uint32_t *urec, const uint64_t *ukey, const uint32_t *uid,
                              const uint32_t *upoff, const uint32_t *table, int np, int part_kind,
                              const GridSpec &pg, uint32_t *ctrl, uint8_t *udead, uint32_t *skybits, uint32_t n_max,
                              int n_wg, hipStream_t s)
{
    const int DP = sky_dp(d);
    const int JB = np <= 256 ? 1 : (np + 255) / 256;
#define M_CASE(X, P)                                                                                       \
    case X:                                                                                                \
        hipLaunchKernelGGL((k_merge_wave<X, P>), dim3(n_wg), dim3(256), 0, s, urec, ukey, upoff, table, np, \
                           JB, part_kind, pg, ctrl, udead);                                                \
        break;
    switch (DP) {
        M_CASE(4, 4) M_CASE(8, 4) M_CASE(12, 2) M_CASE(16, 2) M_CASE(20, 2)
        default: return hipErrorInvalidValue;
    }
#undef M_CASE
    uint32_t blocks = (n_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_merge_finish, dim3(blocks), dim3(SKY_WG), 0, s, udead, uid, ctrl, skybits);
    return hipGetLastError();
}

// ------------------------------------------------------------------ marking
// Single partition: the local skyline is the skyline; set the bits directly.
__global__ __launch_bounds__(SKY_WG) void k_mark(const uint8_t *__restrict__ flag, const uint32_t *__restrict__ ids,
                                                const uint32_t *n_dev, uint32_t *skybits)
{
    const uint32_t n = *n_dev;
    for (uint32_t r = blockIdx.x * SKY_WG + threadIdx.x; r < n; r += gridDim.x * SKY_WG)
        if (flag[r]) {
            const uint32_t id = ids[r];
            atomicOr(&skybits[id >> 5], 1u << (id & 31));
        }
}

hipError_t launch_mark(const uint8_t *flag, const uint32_t *ids, const uint32_t *n_dev, uint32_t n_max,
                       uint32_t *skybits, hipStream_t s)
{
    uint32_t blocks = (n_max + SKY_WG - 1) / SKY_WG;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_mark, dim3(blocks), dim3(SKY_WG), 0, s, flag, ids, n_dev, skybits);
    return hipGetLastError();
}

// Global merge (the final round of Algorithm 2, Sky(u) by SFS): u is re-sorted
// by its (Q, K) key and run through the local-skyline kernel as one partition.
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
