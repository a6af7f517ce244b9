// Dominance tests of wave-uniform records against rows of query points (one
// point per lane and row), shared by the dominance and filter kernels. Device
// code only; included by the .hip sources that run such tests.
#pragma once
#include "sky_internal.h"

// Coordinate words a dominance test compares: d rounded up to even. The words
// from d to DP - 3 are zero in every record and point (the record layout in
// sky_internal.h), so they decide nothing; empty corners and representative
// pads are all-ones in every coordinate word, so they still pass no test. The
// even count keeps two variants per record width.
static inline int sky_nc(int d) { return d + (d & 1); }

// One record r (wave-uniform, held in scalar registers) against the rows: the
// lanes where r dominates the row's point leave am[q] (Def. 1 on the records:
// every coordinate word <=, and the sums K differ). Written here with one lane
// mask per compare; every shape the kernels use (records of 4..20 words, 1..4
// rows) takes the exec-mask specialization further down, which computes the
// same masks.
template <int DP, int NC, int PPL>
__device__ __forceinline__ void test_rec(const uint32_t (&r)[DP], const uint32_t (&x)[PPL][DP - 2],
                                         const uint64_t (&K)[PPL], uint64_t (&am)[PPL])
{
    const uint64_t Kw = ((uint64_t)r[DP - 1] << 32) | r[DP - 2];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        uint64_t dm = __ballot(Kw != K[q]);
#pragma unroll
        for (int k = 0; k < NC; ++k) dm &= __ballot(r[k] <= x[q][k]);
        am[q] &= ~dm;
    }
}

// Mask of the live lanes whose point a corner c is <= in every coordinate.
template <int ND, int NC, int PPL>
__device__ __forceinline__ uint64_t corner_hits(const uint32_t *c, const uint32_t (&x)[PPL][ND],
                                                const uint64_t (&am)[PPL])
{
    uint64_t hit = 0;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        uint64_t t = am[q];
#pragma unroll
        for (int k = 0; k < NC; ++k) t &= __ballot(c[k] <= x[q][k]);
        hit |= t;
    }
    return hit;
}

// ------------------------------------------------------------------ exec-mask chains
// The same tests with the lane masks kept in EXEC: v_cmpx clears the lanes where
// its compare fails, so a chain of them over one row leaves exactly the lanes
// where every compare holds, with no scalar AND per compare (the scalar unit,
// one instruction per SIMD every four cycles, would otherwise issue more than
// the vector unit). Each asm block saves EXEC, runs the chains of all rows,
// folds each chain's result into that row's mask and restores EXEC before it
// ends, so no compiler-generated instruction runs under the narrowed mask.
// The blocks are entered in wave-uniform control flow with every lane active.
// Record words and corners are scalar operands (src0), the point's words
// vector operands.
#define CX_CMP(q, k) "v_cmpx_le_u32_e32 vcc, %[r" #k "], %[x" #q "_" #k "]\n\t"
#define CX_C2(q) CX_CMP(q, 0) CX_CMP(q, 1)
#define CX_C4(q) CX_C2(q) CX_CMP(q, 2) CX_CMP(q, 3)
#define CX_C6(q) CX_C4(q) CX_CMP(q, 4) CX_CMP(q, 5)
#define CX_C8(q) CX_C6(q) CX_CMP(q, 6) CX_CMP(q, 7)
#define CX_C10(q) CX_C8(q) CX_CMP(q, 8) CX_CMP(q, 9)
#define CX_C12(q) CX_C10(q) CX_CMP(q, 10) CX_CMP(q, 11)
#define CX_C14(q) CX_C12(q) CX_CMP(q, 12) CX_CMP(q, 13)
#define CX_C16(q) CX_C14(q) CX_CMP(q, 14) CX_CMP(q, 15)
#define CX_R(k) [r##k] "s"(r[k])
#define CX_R2 CX_R(0), CX_R(1)
#define CX_R4 CX_R2, CX_R(2), CX_R(3)
#define CX_R6 CX_R4, CX_R(4), CX_R(5)
#define CX_R8 CX_R6, CX_R(6), CX_R(7)
#define CX_R10 CX_R8, CX_R(8), CX_R(9)
#define CX_R12 CX_R10, CX_R(10), CX_R(11)
#define CX_R14 CX_R12, CX_R(12), CX_R(13)
#define CX_R16 CX_R14, CX_R(14), CX_R(15)
#define CX_X(q, k) [x##q##_##k] "v"(x[q][k])
#define CX_X2(q) CX_X(q, 0), CX_X(q, 1)
#define CX_X4(q) CX_X2(q), CX_X(q, 2), CX_X(q, 3)
#define CX_X6(q) CX_X4(q), CX_X(q, 4), CX_X(q, 5)
#define CX_X8(q) CX_X6(q), CX_X(q, 6), CX_X(q, 7)
#define CX_X10(q) CX_X8(q), CX_X(q, 8), CX_X(q, 9)
#define CX_X12(q) CX_X10(q), CX_X(q, 10), CX_X(q, 11)
#define CX_X14(q) CX_X12(q), CX_X(q, 12), CX_X(q, 13)
#define CX_X16(q) CX_X14(q), CX_X(q, 14), CX_X(q, 15)
// a record against row q: equal presort keys never dominate, then every coordinate
#define CX_TROW(q, CN)                                                                \
    "s_mov_b64 exec, %[am" #q "]\n\t"                                                 \
    "v_cmpx_ne_u64_e32 vcc, %[kw], %[k" #q "]\n\t" CN(q)                              \
    "s_xor_b64 %[am" #q "], %[am" #q "], exec\n\t"
// a corner against row q: the live lanes it is <= in every coordinate join hit
#define CX_CROW(q, CN) "s_mov_b64 exec, %[am" #q "]\n\t" CN(q) "s_or_b64 %[hit], %[hit], exec\n\t"
#define CX_BEGIN "s_mov_b64 %[sv], exec\n\t"
#define CX_END "s_mov_b64 exec, %[sv]"
#define CX_K(q) [k##q] "v"(K[q])
#define CX_AMI(q) [am##q] "s"(am[q])

#define CX_DEFINE(DPV, NCV, CN, RS, XS)                                                                                  \
    template <>                                                                                                    \
    __device__ __forceinline__ void test_rec<DPV, NCV, 1>(const uint32_t (&r)[DPV], const uint32_t (&x)[1][DPV - 2],   \
                                                        const uint64_t (&K)[1], uint64_t (&am)[1])                 \
    {                                                                                                              \
        const uint64_t Kw = ((uint64_t)r[DPV - 1] << 32) | r[DPV - 2];                                                   \
        uint64_t sv;                                                                                               \
        asm volatile(CX_BEGIN CX_TROW(0, CN) CX_END                                                                \
                     : [sv] "=&s"(sv), [am0] "+s"(am[0])                                                           \
                     : [kw] "s"(Kw), RS, CX_K(0), XS(0)                                                            \
                     : "vcc", "scc");                                                                                     \
    }                                                                                                              \
    template <>                                                                                                    \
    __device__ __forceinline__ void test_rec<DPV, NCV, 2>(const uint32_t (&r)[DPV], const uint32_t (&x)[2][DPV - 2],   \
                                                        const uint64_t (&K)[2], uint64_t (&am)[2])                 \
    {                                                                                                              \
        const uint64_t Kw = ((uint64_t)r[DPV - 1] << 32) | r[DPV - 2];                                                   \
        uint64_t sv;                                                                                               \
        asm volatile(CX_BEGIN CX_TROW(0, CN) CX_TROW(1, CN) CX_END                                                 \
                     : [sv] "=&s"(sv), [am0] "+s"(am[0]), [am1] "+s"(am[1])                                        \
                     : [kw] "s"(Kw), RS, CX_K(0), XS(0), CX_K(1), XS(1)                                            \
                     : "vcc", "scc");                                                                                     \
    }                                                                                                              \
    template <>                                                                                                    \
    __device__ __forceinline__ void test_rec<DPV, NCV, 3>(const uint32_t (&r)[DPV], const uint32_t (&x)[3][DPV - 2],   \
                                                        const uint64_t (&K)[3], uint64_t (&am)[3])                 \
    {                                                                                                              \
        const uint64_t Kw = ((uint64_t)r[DPV - 1] << 32) | r[DPV - 2];                                                   \
        uint64_t sv;                                                                                               \
        asm volatile(CX_BEGIN CX_TROW(0, CN) CX_TROW(1, CN) CX_TROW(2, CN) CX_END                                  \
                     : [sv] "=&s"(sv), [am0] "+s"(am[0]), [am1] "+s"(am[1]), [am2] "+s"(am[2])                     \
                     : [kw] "s"(Kw), RS, CX_K(0), XS(0), CX_K(1), XS(1), CX_K(2), XS(2)                            \
                     : "vcc", "scc");                                                                                     \
    }                                                                                                              \
    template <>                                                                                                    \
    __device__ __forceinline__ void test_rec<DPV, NCV, 4>(const uint32_t (&r)[DPV], const uint32_t (&x)[4][DPV - 2],   \
                                                        const uint64_t (&K)[4], uint64_t (&am)[4])                 \
    {                                                                                                              \
        const uint64_t Kw = ((uint64_t)r[DPV - 1] << 32) | r[DPV - 2];                                                   \
        uint64_t sv;                                                                                               \
        asm volatile(CX_BEGIN CX_TROW(0, CN) CX_TROW(1, CN) CX_TROW(2, CN) CX_TROW(3, CN) CX_END                   \
                     : [sv] "=&s"(sv), [am0] "+s"(am[0]), [am1] "+s"(am[1]), [am2] "+s"(am[2]), [am3] "+s"(am[3])  \
                     : [kw] "s"(Kw), RS, CX_K(0), XS(0), CX_K(1), XS(1), CX_K(2), XS(2), CX_K(3), XS(3)            \
                     : "vcc", "scc");                                                                                     \
    }                                                                                                              \
    template <>                                                                                                    \
    __device__ __forceinline__ uint64_t corner_hits<DPV - 2, NCV, 1>(const uint32_t *r, const uint32_t (&x)[1][DPV - 2],          \
                                                           const uint64_t (&am)[1])                                \
    {                                                                                                              \
        uint64_t sv, hit = 0;                                                                                      \
        asm volatile(CX_BEGIN CX_CROW(0, CN) CX_END                                                                \
                     : [sv] "=&s"(sv), [hit] "+s"(hit)                                                             \
                     : RS, CX_AMI(0), XS(0)                                                                        \
                     : "vcc", "scc");                                                                                     \
        return hit;                                                                                                \
    }                                                                                                              \
    template <>                                                                                                    \
    __device__ __forceinline__ uint64_t corner_hits<DPV - 2, NCV, 2>(const uint32_t *r, const uint32_t (&x)[2][DPV - 2],          \
                                                           const uint64_t (&am)[2])                                \
    {                                                                                                              \
        uint64_t sv, hit = 0;                                                                                      \
        asm volatile(CX_BEGIN CX_CROW(0, CN) CX_CROW(1, CN) CX_END                                                 \
                     : [sv] "=&s"(sv), [hit] "+s"(hit)                                                             \
                     : RS, CX_AMI(0), XS(0), CX_AMI(1), XS(1)                                                      \
                     : "vcc", "scc");                                                                                     \
        return hit;                                                                                                \
    }                                                                                                              \
    template <>                                                                                                    \
    __device__ __forceinline__ uint64_t corner_hits<DPV - 2, NCV, 3>(const uint32_t *r, const uint32_t (&x)[3][DPV - 2],          \
                                                           const uint64_t (&am)[3])                                \
    {                                                                                                              \
        uint64_t sv, hit = 0;                                                                                      \
        asm volatile(CX_BEGIN CX_CROW(0, CN) CX_CROW(1, CN) CX_CROW(2, CN) CX_END                                  \
                     : [sv] "=&s"(sv), [hit] "+s"(hit)                                                             \
                     : RS, CX_AMI(0), XS(0), CX_AMI(1), XS(1), CX_AMI(2), XS(2)                                    \
                     : "vcc", "scc");                                                                                     \
        return hit;                                                                                                \
    }                                                                                                              \
    template <>                                                                                                    \
    __device__ __forceinline__ uint64_t corner_hits<DPV - 2, NCV, 4>(const uint32_t *r, const uint32_t (&x)[4][DPV - 2],          \
                                                           const uint64_t (&am)[4])                                \
    {                                                                                                              \
        uint64_t sv, hit = 0;                                                                                      \
        asm volatile(CX_BEGIN CX_CROW(0, CN) CX_CROW(1, CN) CX_CROW(2, CN) CX_CROW(3, CN) CX_END                   \
                     : [sv] "=&s"(sv), [hit] "+s"(hit)                                                             \
                     : RS, CX_AMI(0), XS(0), CX_AMI(1), XS(1), CX_AMI(2), XS(2), CX_AMI(3), XS(3)                  \
                     : "vcc", "scc");                                                                                     \
        return hit;                                                                                                \
    }

// (record words, compared words): NC = d rounded up to even (sky_nc), at most DP - 2
CX_DEFINE(4, 2, CX_C2, CX_R2, CX_X2)
CX_DEFINE(8, 4, CX_C4, CX_R4, CX_X4)
CX_DEFINE(8, 6, CX_C6, CX_R6, CX_X6)
CX_DEFINE(12, 8, CX_C8, CX_R8, CX_X8)
CX_DEFINE(12, 10, CX_C10, CX_R10, CX_X10)
CX_DEFINE(16, 12, CX_C12, CX_R12, CX_X12)
CX_DEFINE(16, 14, CX_C14, CX_R14, CX_X14)
CX_DEFINE(20, 16, CX_C16, CX_R16, CX_X16)
