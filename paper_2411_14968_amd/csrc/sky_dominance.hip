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

// Next work ticket of a persistent workgroup. Wave 0 takes it under a
// wave-uniform branch: all 64 lanes add 1 (the counter advances by 64 per
// ticket), so no lane-divergent region sits at the head or the backedge of the
// loops that call this. A divergent `if (threadIdx.x == 0)` there lets the
// compiler rotate the loop into a divergent backedge, and lanes then wait at a
// barrier for a lane that never comes back: a deadlock.
__device__ __forceinline__ uint32_t block_ticket(uint32_t *counter, uint32_t *s_g)
{
    if (__builtin_amdgcn_readfirstlane(threadIdx.x) == 0) {
        const uint32_t v = atomicAdd(counter, 1u);
        *s_g = __builtin_amdgcn_readfirstlane(v) >> 6;
    }
    __syncthreads();
    const uint32_t g = __builtin_amdgcn_readfirstlane(*s_g);
    __syncthreads();
    return g;
}

// ------------------------------------------------------------------ local skyline
// Persistent workgroups take chunks (LS_WG * PPL consecutive points of one
// partition) from a ticket counter. A point of chunk c is in the local skyline
// u_j iff no earlier point of the partition dominates it. It is tested
//  1. against each earlier chunk c' < c: the compacted local skyline of c' if
//     c' has been published, else all raw points of c' (testing against every
//     earlier point is exact too, since a dominated dominator is itself
//     dominated by an earlier skyline point) -- so no workgroup ever waits;
//  2. against the earlier points of its own chunk that survived step 1 (a
//     dominator killed in step 1 was killed by a point that also dominates).
// The chunk then publishes its skyline points, compacted in key order, with a
// release store of (count + 1) to its state word.
template <int DP, int PPL>
__global__ __launch_bounds__(LS_WG) void k_local_sky(const uint32_t *__restrict__ raw, uint32_t *win,
                                                    uint32_t *wpos, uint32_t *state,
                                                    const uint32_t *__restrict__ poff,
                                                    const uint32_t *__restrict__ st_off,
                                                    const uint32_t *__restrict__ table, uint32_t *ctrl,
                                                    int ticket_slot, int nchunk_slot, uint8_t *in_u)
{
    constexpr int B = LS_WG * PPL, ND = DP - 2;
    __shared__ __attribute__((aligned(16))) uint32_t s_tile[4][64 * DP];
    __shared__ __attribute__((aligned(16))) uint32_t s_chunk[B * DP];
    __shared__ uint8_t s_alive[B];
    __shared__ uint32_t s_cnt[PPL][4];
    __shared__ uint32_t s_g;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t nchunks = __builtin_amdgcn_readfirstlane(ctrl[nchunk_slot]);
    uint32_t *tile = s_tile[wv];
    for (;;) {
        const uint32_t g = block_ticket(&ctrl[ticket_slot], &s_g);
        if (g >= nchunks) break;
        const uint32_t j = __builtin_amdgcn_readfirstlane(table[2 * g]);
        const uint32_t c = __builtin_amdgcn_readfirstlane(table[2 * g + 1]);
        const uint32_t pbeg = poff[j], pend = poff[j + 1];
        const uint32_t start = pbeg + c * B;
        const uint32_t len = min((uint32_t)B, pend - start);
        uint32_t x[PPL][ND];
        uint64_t K[PPL];
        bool al[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const uint32_t o = q * LS_WG + t;
            al[q] = o < len;
            const uint4 *s = reinterpret_cast<const uint4 *>(raw + (size_t)(start + (al[q] ? o : 0)) * DP);
            uint32_t w[DP];
#pragma unroll
            for (int k = 0; k < DP / 4; ++k) {
                const uint4 v = s[k];
                w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int k = 0; k < ND; ++k) x[q][k] = w[k];
            K[q] = ((uint64_t)w[DP - 1] << 32) | w[DP - 2];
        }
        // 1. earlier chunks of the partition, strongest (smallest keys) first
        const uint32_t sbase = st_off[j];
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
        // 2. earlier survivors of the own chunk
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const uint32_t o = q * LS_WG + t;
            s_alive[o] = al[q] ? 1 : 0;
            if (o < len) {
                uint4 *d = reinterpret_cast<uint4 *>(s_chunk + o * DP);
                uint32_t w[DP];
#pragma unroll
                for (int k = 0; k < ND; ++k) w[k] = x[q][k];
                w[DP - 2] = (uint32_t)K[q];
                w[DP - 1] = (uint32_t)(K[q] >> 32);
#pragma unroll
                for (int k = 0; k < DP / 4; ++k) d[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
            }
        }
        __syncthreads();
        {
            const uint32_t wend = min(len, (uint32_t)((PPL - 1) * LS_WG + wv * 64 + 64));
            for (uint32_t w = 0; w < wend; ++w) {
                if ((w & 7) == 0 && !__any(any_alive<PPL>(al))) break;
                if (!s_alive[w]) continue;
                const uint32_t *r = s_chunk + w * DP;
                bool keep[PPL];
#pragma unroll
                for (int q = 0; q < PPL; ++q) keep[q] = true;
                test_rec<DP, PPL>(r, x, K, keep);
#pragma unroll
                for (int q = 0; q < PPL; ++q)
                    if (w < (uint32_t)(q * LS_WG) + t) al[q] = al[q] && keep[q];
            }
        }
        // publish: flags, then the compacted records in key order
        uint32_t tot = 0, rank[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const uint32_t o = q * LS_WG + t;
            if (o < len) in_u[start + o] = al[q] ? 1 : 0;
            const uint64_t m = __ballot(al[q]);
            rank[q] = (uint32_t)__popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull));
            if (lane == 0) s_cnt[q][wv] = (uint32_t)__popcll(m);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            uint32_t base = tot;
            for (uint32_t w = 0; w < 4; ++w) {
                if (w < wv) base += s_cnt[q][w];
                tot += s_cnt[q][w];
            }
            rank[q] += base;
        }
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            if (al[q]) {
                const uint32_t o = q * LS_WG + t;
                uint4 *d = reinterpret_cast<uint4 *>(win + (size_t)(start + rank[q]) * DP);
                const uint4 *s = reinterpret_cast<const uint4 *>(s_chunk + o * DP);
#pragma unroll
                for (int k = 0; k < DP / 4; ++k) d[k] = s[k];
                wpos[start + rank[q]] = start + o;
            }
        }
        __threadfence();
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(t) == 0)   // all lanes of wave 0 store the same value
            __hip_atomic_store(&state[sbase + c], tot + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int PPL>
static hipError_t local_sky_ppl(int DP, const uint32_t *raw, uint32_t *win, uint32_t *wpos, uint32_t *state,
                                const uint32_t *poff, const uint32_t *st_off, const uint32_t *table,
                                uint32_t *ctrl, int ticket_slot, int nchunk_slot, uint8_t *in_u, int n_wg,
                                hipStream_t s)
{
#define L_CASE(X)                                                                                      \
    case X:                                                                                            \
        hipLaunchKernelGGL((k_local_sky<X, PPL>), dim3(n_wg), dim3(LS_WG), 0, s, raw, win, wpos, state, \
                           poff, st_off, table, ctrl, ticket_slot, nchunk_slot, in_u);                 \
        break;
    switch (DP) {
        L_CASE(4) L_CASE(8) L_CASE(12) L_CASE(16) L_CASE(20)
        default: return hipErrorInvalidValue;
    }
#undef L_CASE
    return hipGetLastError();
}

int local_sky_chunk(int d)
{
    return sky_dp(d) <= 8 ? LS_WG * 4 : LS_WG * 2;
}

hipError_t launch_local_sky(int d, const uint32_t *raw, uint32_t *win, uint32_t *wpos, uint32_t *state,
                            const uint32_t *poff, const uint32_t *st_off, const uint32_t *table, uint32_t *ctrl,
                            int ticket_slot, int nchunk_slot, uint8_t *in_u, int n_wg, hipStream_t s)
{
    const int DP = sky_dp(d);
    if (DP <= 8)
        return local_sky_ppl<4>(DP, raw, win, wpos, state, poff, st_off, table, ctrl, ticket_slot, nchunk_slot,
                                in_u, n_wg, s);
    return local_sky_ppl<2>(DP, raw, win, wpos, state, poff, st_off, table, ctrl, ticket_slot, nchunk_slot,
                            in_u, n_wg, s);
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
// dominate, and u_j is sorted by that key, so each u_j is scanned up to the
// largest key of the wave's points. Survivors set their bit in the skyline
// bitmap of original ids.
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
__global__ __launch_bounds__(LS_WG) void k_merge_noseq(const uint32_t *__restrict__ urec,
                                                      const uint64_t *__restrict__ ukey,
                                                      const uint32_t *__restrict__ uid,
                                                      const uint32_t *__restrict__ upoff,
                                                      const uint32_t *__restrict__ table, int np, int part_kind,
                                                      GridSpec pg, uint32_t *ctrl, uint32_t *skybits)
{
    constexpr int B = LS_WG * PPL, ND = DP - 2;
    __shared__ __attribute__((aligned(16))) uint32_t s_tile[4][64 * DP];
    __shared__ uint32_t s_g;
    const uint32_t t = threadIdx.x, wv = t >> 6;
    const uint32_t nchunks = __builtin_amdgcn_readfirstlane(ctrl[C_NCHUNK2]);
    uint32_t *tile = s_tile[wv];
    for (;;) {
        const uint32_t g = block_ticket(&ctrl[C_TICKET2], &s_g);
        if (g >= nchunks) break;
        const uint32_t i = __builtin_amdgcn_readfirstlane(table[2 * g]);
        const uint32_t c = __builtin_amdgcn_readfirstlane(table[2 * g + 1]);
        const uint32_t start = upoff[i] + c * B;
        const uint32_t len = min((uint32_t)B, upoff[i + 1] - start);
        uint32_t x[PPL][ND];
        uint64_t K[PPL];
        bool al[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const uint32_t o = q * LS_WG + t;
            al[q] = o < len;
            const uint4 *s = reinterpret_cast<const uint4 *>(urec + (size_t)(start + (al[q] ? o : 0)) * DP);
            uint32_t w[DP];
#pragma unroll
            for (int k = 0; k < DP / 4; ++k) {
                const uint4 v = s[k];
                w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int k = 0; k < ND; ++k) x[q][k] = w[k];
            K[q] = ((uint64_t)w[DP - 1] << 32) | w[DP - 2];
        }
        // largest presort key among the wave's points (points are key-sorted)
        uint32_t last = (uint32_t)((PPL - 1) * LS_WG) + wv * 64 + 63;
        if (last >= len) last = len ? len - 1 : 0;
        const uint64_t kmax = ukey[start + last];
        for (int jj = 0; jj < np; ++jj) {
            if (!__any(any_alive<PPL>(al))) break;
            const uint32_t jp = (uint32_t)jj;
            bool pd;
            if (part_kind == P_SLICED) pd = jp < i;
            else if (part_kind == P_GRID) pd = jp != i && grid_weakly_below(jp, i, pg);
            else pd = jp != i;
            if (!pd) continue;
            uint32_t lo = upoff[jp], hi = upoff[jp + 1];
            // first position with key > kmax
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (ukey[mid] <= kmax) lo = mid + 1; else hi = mid;
            }
            scan_records<DP, PPL>(urec + (size_t)upoff[jp] * DP, lo - upoff[jp], tile, x, K, al);
        }
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            if (al[q]) {
                const uint32_t id = uid[start + q * LS_WG + t];
                atomicOr(&skybits[id >> 5], 1u << (id & 31));
            }
        }
        __syncthreads();   // the loop body ends converged (see block_ticket)
    }
}

hipError_t launch_merge_noseq(int d, const uint32_t *urec, const uint64_t *ukey, const uint32_t *uid,
                              const uint32_t *upoff, const uint32_t *table, int np, int part_kind,
                              const GridSpec &pg, uint32_t *ctrl, uint32_t *skybits, int n_wg, hipStream_t s)
{
    const int DP = sky_dp(d);
#define M_CASE(X, P)                                                                                      \
    case X:                                                                                               \
        hipLaunchKernelGGL((k_merge_noseq<X, P>), dim3(n_wg), dim3(LS_WG), 0, s, urec, ukey, uid, upoff,    \
                           table, np, part_kind, pg, ctrl, skybits);                                      \
        break;
    switch (DP) {
        M_CASE(4, 4) M_CASE(8, 4) M_CASE(12, 2) M_CASE(16, 2) M_CASE(20, 2)
        default: return hipErrorInvalidValue;
    }
#undef M_CASE
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
