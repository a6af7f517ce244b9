// Learned scorer for representatives and presort order: a monotone MLP
// g(x) = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with W1, W2, w3 >= 0, so g is
// non-decreasing in every coordinate and sorting by g is a topological sort
// with respect to dominance (Section 2). It plays the role of the monotone
// scoring function of Algorithm 1 and of the dominance-region score of
// Section 4.1, fitted to the data. Also the dominance-count kernel (Def. 2)
// that produces its training targets.
//
// Inference: bfloat16 inputs and weights, float32 accumulation on MFMA
// (v_mfma_f32_16x16x32_bf16), the first hidden layer rounded to bfloat16;
// points are staged through LDS one tile per workgroup.
// Training: float32 VALU forward/backward with the same rounding points,
// per-workgroup gradient partials reduced in a fixed order, Adam on float32
// master weights, projection of the weight matrices onto >= 0.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include <string>

#include "../../include/skyline.h"
#include "sky_internal.h"
#include "sky_mlp.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define MLP_H 64

struct sky_mlp {
    int device = 0;
    int d = 0, h = MLP_H;
    int64_t np = 0;
    int64_t step = 0;
    float *P = nullptr, *m = nullptr, *v = nullptr;    // master parameters and Adam moments
    bf16x8 *A1 = nullptr, *A2 = nullptr;                // packed MFMA operands
    f32x4 *C1 = nullptr, *C2 = nullptr, *W3 = nullptr;
    float *b3 = nullptr;
    float *partial = nullptr;                            // gradient partials
    int64_t partial_cap = 0;
    float *grad = nullptr, *loss = nullptr;
    uint64_t serial = 0;                                 // unique per model of the process
};

int sky_mlp_dim(const sky_mlp *m) { return m ? m->d : -1; }
uint64_t sky_mlp_serial(const sky_mlp *m) { return m ? m->serial : 0; }

static std::atomic<uint64_t> g_mlp_serial{0};

extern "C" int64_t sky_mlp_nparams(int32_t d, int32_t h)
{
    return (int64_t)h * d + h + (int64_t)h * h + h + h + 1;
}

// Offsets of the parameter blocks in the flat layout.
struct MlpLayout {
    int d, h;
    __host__ __device__ int W1() const { return 0; }
    __host__ __device__ int b1() const { return h * d; }
    __host__ __device__ int W2() const { return h * d + h; }
    __host__ __device__ int b2() const { return h * d + h + h * h; }
    __host__ __device__ int w3() const { return h * d + 2 * h + h * h; }
    __host__ __device__ int b3() const { return h * d + 3 * h + h * h; }
};

__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

// relu as one integer max on the bits: a float with the sign bit clear is a
// non-negative int and stays, any other becomes +0. Equal to max(x, 0) for every
// non-NaN x (-0 gives +0); fmaxf would add a canonicalising max per value.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// ------------------------------------------------------------------ operand packing
// MFMA 16x16x32: lane l = 16 g + r holds row r of A (K slots 8g..8g+7) and
// column r of B (same K slots); D row 4g + i, column r for i < 4.
// Layer 1: A = W1 tile (rows = hidden units 16 mt + r, K = input dims 8g + j).
// Layer 2: K slot (step s, group g, element j) stands for hidden unit
//   u = 16 (2 s + j / 4) + 4 g + j % 4,
// exactly the units that lane (g, p) holds in layer 1's D, so the first
// hidden layer never leaves the lane.
__global__ void k_mlp_pack(const float *__restrict__ P, int d, bf16x8 *A1, bf16x8 *A2, f32x4 *C1, f32x4 *C2,
                           f32x4 *W3, float *b3)
{
    const MlpLayout L{d, MLP_H};
    const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
    for (int mt = 0; mt < 4; ++mt) {
        bf16x8 a;
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            a[j] = (__bf16)(k < d ? P[L.W1() + (16 * mt + r) * d + k] : 0.0f);
        }
        A1[mt * 64 + l] = a;
        f32x4 c1, c2, w3;
        for (int i = 0; i < 4; ++i) {
            const int u = 16 * mt + 4 * g + i;
            c1[i] = P[L.b1() + u];
            c2[i] = P[L.b2() + u];
            w3[i] = bf16_round(P[L.w3() + u]);
        }
        C1[mt * 64 + l] = c1;
        C2[mt * 64 + l] = c2;
        W3[mt * 64 + l] = w3;
        for (int s = 0; s < 2; ++s) {
            bf16x8 a2;
            for (int j = 0; j < 8; ++j) {
                const int u = 16 * (2 * s + j / 4) + 4 * g + (j % 4);
                a2[j] = (__bf16)P[L.W2() + (16 * mt + r) * MLP_H + u];
            }
            A2[(mt * 2 + s) * 64 + l] = a2;
        }
    }
    if (threadIdx.x == 0) *b3 = P[L.b3()];
}

// ------------------------------------------------------------------ inference (MFMA)
// A workgroup scores MLP_TILE consecutive points: their coordinates go to LDS
// first, with every load of the tile issued before any is used (KD rows per
// point, rows past d repeat row d - 1 and are not read), then each wave runs
// MFMA passes of 16 points from LDS. One load round trip per tile instead of
// one per pass.
#define MLP_TILE 512
template <int KD>
__global__ __launch_bounds__(256, 4) void k_mlp_score(const float *__restrict__ pts, uint32_t n, int d,
                                                   const bf16x8 *__restrict__ A1, const bf16x8 *__restrict__ A2,
                                                   const f32x4 *__restrict__ C1, const f32x4 *__restrict__ C2,
                                                   const f32x4 *__restrict__ W3, const float *__restrict__ b3p,
                                                   float *__restrict__ out)
{
    constexpr int PPT = MLP_TILE / 256;   // points per thread in the tile load
    __shared__ float s_x[KD][MLP_TILE];
    const int l = threadIdx.x & 63, g = l >> 4, p = l & 15, wv = threadIdx.x >> 6;
    const uint32_t base = blockIdx.x * MLP_TILE;
    {
        float v[PPT][KD];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const uint32_t pt = base + q * 256 + threadIdx.x, ptc = pt < n ? pt : n - 1;
#pragma unroll
            for (int k = 0; k < KD; ++k) v[q][k] = pts[(size_t)(k < d ? k : d - 1) * n + ptc];
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q)
#pragma unroll
            for (int k = 0; k < KD; ++k) s_x[k][q * 256 + threadIdx.x] = v[q][k];
    }
    bf16x8 a1[4], a2[8];
    f32x4 c1[4], c2[4], w3[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        a1[mt] = A1[mt * 64 + l];
        c1[mt] = C1[mt * 64 + l];
        c2[mt] = C2[mt * 64 + l];
        w3[mt] = W3[mt * 64 + l];
        a2[2 * mt] = A2[(2 * mt) * 64 + l];
        a2[2 * mt + 1] = A2[(2 * mt + 1) * 64 + l];
    }
    const float b3 = *b3p;
    __syncthreads();
    for (int it = wv; it < MLP_TILE / 16; it += 4) {
        const uint32_t lp = it * 16 + p, pt = base + lp;
        bf16x8 bx;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            const float xv = s_x[k < KD ? k : KD - 1][lp];   // in bounds for every lane: no branch
            bx[j] = (__bf16)((k < d && pt < n) ? xv : 0.0f);
        }
        f32x4 z1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) z1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[mt], bx, c1[mt], 0, 0, 0);
        bf16x8 h1[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) h1[s][j] = (__bf16)relu(z1[2 * s + j / 4][j % 4]);
        float acc = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 z2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[2 * mt], h1[0], c2[mt], 0, 0, 0);
            z2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[2 * mt + 1], h1[1], z2, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc = fmaf(w3[mt][i], relu(z2[i]), acc);
        }
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        if (g == 0 && pt < n) out[pt] = acc + b3;
    }
}

int sky_mlp_score_internal(const sky_mlp *m, const float *pts, uint32_t n, int d, float *out, hipStream_t s)
{
    if (!m || m->d != d) return SKY_ERR_MODEL;
    if (n == 0) return SKY_OK;
    const uint32_t blocks = (n + MLP_TILE - 1) / MLP_TILE;
    if (d <= 8)
        hipLaunchKernelGGL(k_mlp_score<8>, dim3(blocks), dim3(256), 0, s, pts, n, d, m->A1, m->A2, m->C1, m->C2,
                           m->W3, m->b3, out);
    else
        hipLaunchKernelGGL(k_mlp_score<16>, dim3(blocks), dim3(256), 0, s, pts, n, d, m->A1, m->A2, m->C1, m->C2,
                           m->W3, m->b3, out);
    return hipGetLastError() == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

// ------------------------------------------------------------------ training (VALU)
// A workgroup of four waves walks chunks of 64 consecutive points, one point per
// lane; wave w owns hidden units [16w, 16w + 16) of both layers. Forward and
// backward use the inference rounding points (bfloat16 inputs, weights and first
// hidden layer; the roundings count as identity in the backward pass). A chunk's
// activations pass between the waves through LDS (rows padded to 65 words, so
// that row-per-lane and column-per-lane accesses both avoid bank conflicts); the
// gradient sums stay in registers across the workgroup's chunks and are written
// once, as the workgroup's partial. About 75 KB of LDS: two workgroups, eight
// waves, per CU.
#define TR_P 64                    // points per chunk, one per lane
#define TR_WAVES 4
#define TR_J (MLP_H / TR_WAVES)    // hidden units per wave
#define TR_S (MLP_H + 1)           // padded row stride of the per-point rows
#define TR_XS (SKY_MAXD + 1)       // padded row stride of the inputs
#define TR_MAXWG 512               // workgroups per launch at most (two per CU)

// One halving exchange: lanes with bit M set keep the upper H of the first 2H
// values, the others the lower H, each adding the partner lane's copy.
template <int H, int M>
__device__ __forceinline__ void halve(float (&v)[TR_J], int l)
{
    const bool up = (l & M) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float keep = up ? v[i + H] : v[i], send = up ? v[i] : v[i + H];
        v[i] = keep + __shfl_xor(send, M, 64);
    }
}

// Totals over the 64 lanes of a wave of v[0..15], by halving exchanges: on
// return lane l holds the total of index l >> 2.
__device__ __forceinline__ float wave_sum16(float (&v)[TR_J], int l)
{
    halve<8, 32>(v, l);
    halve<4, 16>(v, l);
    halve<2, 8>(v, l);
    halve<1, 4>(v, l);
    float a = v[0];
    a += __shfl_xor(a, 2, 64);
    a += __shfl_xor(a, 1, 64);
    return a;
}

__device__ __forceinline__ float wave_sum(float a)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
}

template <int KD>
__global__ __launch_bounds__(TR_P * TR_WAVES, 2) void k_mlp_fwd_bwd(
    const float *__restrict__ P, const float *__restrict__ pts, uint32_t n_stride, uint32_t first, uint32_t count,
    int d, const float *__restrict__ y, float inv_n, float *__restrict__ partial, int64_t np,
    float *__restrict__ loss_partial)
{
    const MlpLayout L{d, MLP_H};
    __shared__ __align__(16) float sW2[MLP_H * MLP_H];
    __shared__ __align__(16) float sdz2[MLP_H * TR_P];   // [unit][point]
    __shared__ __align__(16) float sW1[MLP_H * KD];      // zero beyond d
    __shared__ float sb1[MLP_H], sb2[MLP_H], sw3[MLP_H], sg[TR_WAVES][TR_P];
    __shared__ float sx[TR_P * TR_XS], sh1[TR_P * TR_S], sdz1[TR_P * TR_S];   // [point][.]
    const int t = threadIdx.x, l = t & 63, w = t >> 6, j0 = w * TR_J;
    for (int i = t; i < MLP_H * KD; i += TR_P * TR_WAVES) {
        const int j = i / KD, k = i % KD;
        sW1[i] = k < d ? bf16_round(P[L.W1() + j * d + k]) : 0.0f;
    }
    for (int i = t; i < MLP_H * MLP_H; i += TR_P * TR_WAVES) sW2[i] = bf16_round(P[L.W2() + i]);
    if (t < MLP_H) {
        sb1[t] = P[L.b1() + t];
        sb2[t] = P[L.b2() + t];
        sw3[t] = bf16_round(P[L.w3() + t]);
    }
    const float b3 = P[L.b3()];
    constexpr int R1 = MLP_H * KD / (TR_P * TR_WAVES);   // first-layer weight gradients per thread
    float g2[TR_J], gb1[TR_J], gb2[TR_J], gw3[TR_J], g1[R1];
#pragma unroll
    for (int i = 0; i < TR_J; ++i) g2[i] = gb1[i] = gb2[i] = gw3[i] = 0.0f;
#pragma unroll
    for (int i = 0; i < R1; ++i) g1[i] = 0.0f;
    float gb3 = 0.0f, gl = 0.0f;
    const uint32_t nch = (count + TR_P - 1) / TR_P;
    for (uint32_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        __syncthreads();   // weights staged; the previous chunk's sums have read its rows
        const uint32_t idx = ch * TR_P + l;
        const bool valid = idx < count;
        const uint32_t pt = first + (valid ? idx : 0);
        float x[KD];
#pragma unroll
        for (int k = 0; k < KD; ++k) x[k] = (valid && k < d) ? bf16_round(pts[(size_t)k * n_stride + pt]) : 0.0f;
        if (w == 0) {
#pragma unroll
            for (int k = 0; k < KD; ++k) sx[l * TR_XS + k] = x[k];
        }
        // first layer, this wave's units
        uint32_t m1 = 0;
#pragma unroll
        for (int i = 0; i < TR_J; ++i) {
            const int j = j0 + i;
            float z = 0.0f;
#pragma unroll
            for (int k = 0; k < KD; ++k) z = fmaf(sW1[j * KD + k], x[k], z);
            z += sb1[j];
            m1 |= (z > 0.0f ? 1u : 0u) << i;
            sh1[l * TR_S + j] = bf16_round(fmaxf(z, 0.0f));
        }
        __syncthreads();
        // second layer and this wave's share of the output
        float z2[TR_J];
#pragma unroll
        for (int i = 0; i < TR_J; ++i) z2[i] = 0.0f;
#pragma unroll 2
        for (int k = 0; k < MLP_H; k += 4) {
            float hq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) hq[q] = sh1[l * TR_S + k + q];
#pragma unroll
            for (int i = 0; i < TR_J; ++i) {
                const float4 wv = *reinterpret_cast<const float4 *>(&sW2[(j0 + i) * MLP_H + k]);
                z2[i] = fmaf(wv.x, hq[0], z2[i]);
                z2[i] = fmaf(wv.y, hq[1], z2[i]);
                z2[i] = fmaf(wv.z, hq[2], z2[i]);
                z2[i] = fmaf(wv.w, hq[3], z2[i]);
            }
        }
        uint32_t m2 = 0;
        float h2[TR_J], gs = 0.0f;
#pragma unroll
        for (int i = 0; i < TR_J; ++i) {
            const int j = j0 + i;
            const float z = z2[i] + sb2[j];
            h2[i] = fmaxf(z, 0.0f);
            m2 |= (z > 0.0f ? 1u : 0u) << i;
            gs = fmaf(sw3[j], h2[i], gs);
        }
        sg[w][l] = gs;
        __syncthreads();
        const float gval = ((sg[0][l] + sg[1][l]) + (sg[2][l] + sg[3][l])) + b3;
        const float e = valid ? gval - y[pt] : 0.0f;
        const float dg = 2.0f * e * inv_n;
#pragma unroll
        for (int i = 0; i < TR_J; ++i) {
            const int j = j0 + i;
            const float dz = (m2 >> i & 1u) ? dg * sw3[j] : 0.0f;
            sdz2[j * TR_P + l] = dz;
            gb2[i] += dz;
            gw3[i] = fmaf(dg, h2[i], gw3[i]);
        }
        gb3 += dg;   // the same in every wave
        gl = fmaf(e, e, gl);
        __syncthreads();
        // back through the second layer to this wave's first-layer units
        float a[TR_J];
#pragma unroll
        for (int i = 0; i < TR_J; ++i) a[i] = 0.0f;
#pragma unroll 4
        for (int j = 0; j < MLP_H; ++j) {
            const float dz = sdz2[j * TR_P + l];
#pragma unroll
            for (int i4 = 0; i4 < TR_J; i4 += 4) {
                const float4 wv = *reinterpret_cast<const float4 *>(&sW2[j * MLP_H + j0 + i4]);
                a[i4] = fmaf(wv.x, dz, a[i4]);
                a[i4 + 1] = fmaf(wv.y, dz, a[i4 + 1]);
                a[i4 + 2] = fmaf(wv.z, dz, a[i4 + 2]);
                a[i4 + 3] = fmaf(wv.w, dz, a[i4 + 3]);
            }
        }
#pragma unroll
        for (int i = 0; i < TR_J; ++i) {
            const float dz1 = (m1 >> i & 1u) ? a[i] : 0.0f;
            sdz1[l * TR_S + j0 + i] = dz1;
            gb1[i] += dz1;
        }
        __syncthreads();
        // second-layer weight gradients: unit j0 + i, input l, summed over the chunk
#pragma unroll 2
        for (int p = 0; p < TR_P; p += 4) {
            float hq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) hq[q] = sh1[(p + q) * TR_S + l];
#pragma unroll
            for (int i = 0; i < TR_J; ++i) {
                const float4 dz = *reinterpret_cast<const float4 *>(&sdz2[(j0 + i) * TR_P + p]);
                g2[i] = fmaf(dz.x, hq[0], g2[i]);
                g2[i] = fmaf(dz.y, hq[1], g2[i]);
                g2[i] = fmaf(dz.z, hq[2], g2[i]);
                g2[i] = fmaf(dz.w, hq[3], g2[i]);
            }
        }
        // first-layer weight gradients: q = t + 256 rr, unit q / KD, input q % KD
#pragma unroll
        for (int rr = 0; rr < R1; ++rr) {
            const int q = t + rr * TR_P * TR_WAVES, k = q / KD, c = q % KD;
            float acc = g1[rr];
#pragma unroll 8
            for (int p = 0; p < TR_P; ++p) acc = fmaf(sdz1[p * TR_S + k], sx[p * TR_XS + c], acc);
            g1[rr] = acc;
        }
    }
    float *out = partial + (size_t)blockIdx.x * np;
#pragma unroll
    for (int i = 0; i < TR_J; ++i) out[L.W2() + (j0 + i) * MLP_H + l] = g2[i];
#pragma unroll
    for (int rr = 0; rr < R1; ++rr) {
        const int q = t + rr * TR_P * TR_WAVES, k = q / KD, c = q % KD;
        if (c < d) out[L.W1() + k * d + c] = g1[rr];
    }
    const float s1 = wave_sum16(gb1, l), s2 = wave_sum16(gb2, l), s3 = wave_sum16(gw3, l);
    if ((l & 3) == 0) {
        out[L.b1() + j0 + (l >> 2)] = s1;
        out[L.b2() + j0 + (l >> 2)] = s2;
        out[L.w3() + j0 + (l >> 2)] = s3;
    }
    const float sb3 = wave_sum(gb3), sl = wave_sum(gl);
    if (t == 0) {
        out[L.b3()] = sb3;
        loss_partial[blockIdx.x] = sl;
    }
}

// grad[q] = sum over workgroups in order; loss = sum of partials * inv_n.
__global__ void k_mlp_reduce(const float *__restrict__ partial, int nwg, int64_t np, float *grad,
                             const float *__restrict__ loss_partial, float inv_n, float *loss)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < np; q += (int64_t)gridDim.x * blockDim.x) {
        float a = 0.0f;
        for (int w = 0; w < nwg; ++w) a += partial[(size_t)w * np + q];
        grad[q] = a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float a = 0.0f;
        for (int w = 0; w < nwg; ++w) a += loss_partial[w];
        *loss = a * inv_n;
    }
}

// Adam (Kingma & Ba) with bias correction c1 = 1 - beta1^t, c2 = 1 - beta2^t,
// then projection of W1, W2, w3 onto >= 0 (biases stay free).
__global__ void k_mlp_adam(float *P, float *m, float *v, const float *__restrict__ grad, int d, int64_t np, float lr,
                           float beta1, float beta2, float eps, float c1, float c2)
{
    const MlpLayout L{d, MLP_H};
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < np; q += (int64_t)gridDim.x * blockDim.x) {
        const float gq = grad[q];
        const float mq = beta1 * m[q] + (1.0f - beta1) * gq;
        const float vq = beta2 * v[q] + (1.0f - beta2) * gq * gq;
        m[q] = mq;
        v[q] = vq;
        float w = P[q] - lr * (mq / c1) / (sqrtf(vq / c2) + eps);
        const bool is_w = q < L.b1() || (q >= L.W2() && q < L.b2()) || (q >= L.w3() && q < L.b3());
        if (is_w && w < 0.0f) w = 0.0f;
        P[q] = w;
    }
}

__global__ void k_project(float *P, int d, int64_t np)
{
    const MlpLayout L{d, MLP_H};
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < np; q += (int64_t)gridDim.x * blockDim.x) {
        const bool is_w = q < L.b1() || (q >= L.W2() && q < L.b2()) || (q >= L.w3() && q < L.b3());
        if (is_w && P[q] < 0.0f) P[q] = 0.0f;
    }
}

// ------------------------------------------------------------------ dominance counts
// out[i] = #{ j : point i dominates sample point sample[j] } (Def. 2: the
// sample points inside the dominance region of i). The sample is staged in
// LDS as records; each lane counts for its point, no early exit.
template <int DP>
__global__ __launch_bounds__(SKY_WG) void k_domcount(const float *__restrict__ pts, uint32_t n, int d,
                                                    const uint32_t *__restrict__ sample, uint32_t m_host,
                                                    const uint32_t *__restrict__ m_dev, int reverse,
                                                    uint32_t *__restrict__ out)
{
    constexpr int ND = DP - 2;
    const uint32_t m = m_dev ? *m_dev : m_host;   // a count produced on the device needs no host round trip
    __shared__ __attribute__((aligned(16))) uint32_t s_rec[SKY_WG * DP];
    for (uint32_t base = blockIdx.x * SKY_WG; base < n; base += gridDim.x * SKY_WG) {
        const uint32_t i = base + threadIdx.x;
        uint32_t x[ND];
        uint64_t K = 0;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            x[k] = (k < d && i < n) ? ordmap(pts[(size_t)k * n + i]) : 0u;
            K += x[k];
        }
        uint32_t cnt = 0;
        for (uint32_t s0 = 0; s0 < m; s0 += SKY_WG) {
            __syncthreads();
            const uint32_t sj = s0 + threadIdx.x;
            if (sj < m) {
                const uint32_t id = sample[sj];
                uint64_t Ks = 0;
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    const uint32_t w = (k < d && id < n) ? ordmap(pts[(size_t)k * n + id]) : 0u;
                    s_rec[threadIdx.x * DP + k] = w;
                    Ks += w;
                }
                s_rec[threadIdx.x * DP + DP - 2] = (uint32_t)Ks;
                s_rec[threadIdx.x * DP + DP - 1] = (uint32_t)(Ks >> 32);
            }
            __syncthreads();
            const uint32_t ns = min((uint32_t)SKY_WG, m - s0);
            for (uint32_t w = 0; w < ns; ++w) {
                const uint32_t *r = s_rec + w * DP;
                bool dm = true;
                if (reverse) {
#pragma unroll
                    for (int k = 0; k < ND; ++k) dm &= r[k] <= x[k];
                } else {
#pragma unroll
                    for (int k = 0; k < ND; ++k) dm &= x[k] <= r[k];
                }
                const uint64_t Kr = ((uint64_t)r[DP - 1] << 32) | r[DP - 2];
                cnt += (dm && Kr != K) ? 1u : 0u;
            }
        }
        if (i < n) out[i] = cnt;
    }
}

// ------------------------------------------------------------------ training targets
// Residual sample: the sample points that no point of reps dominates (what the
// representatives already prune is left out of the targets). One lane per
// sample point; the kept ids are appended through one counter, so their order
// varies, which no count depends on.
__global__ __launch_bounds__(SKY_WG) void k_residual(const float *__restrict__ pts, uint32_t n, int d,
                                                    const uint32_t *__restrict__ sample, uint32_t m,
                                                    const uint32_t *__restrict__ reps, uint32_t nreps,
                                                    uint32_t *__restrict__ res, uint32_t *__restrict__ kept)
{
    const uint32_t j = blockIdx.x * SKY_WG + threadIdx.x;
    if (j >= m) return;
    const uint32_t t = sample[j];
    uint32_t x[SKY_MAXD];
    uint64_t K = 0;
    for (int k = 0; k < d; ++k) {
        x[k] = ordmap(pts[(size_t)k * n + t]);
        K += x[k];
    }
    bool pruned = false;
    for (uint32_t r = 0; r < nreps && !pruned; ++r) {
        const uint32_t id = reps[r];
        bool le = true;
        uint64_t Kr = 0;
        for (int k = 0; k < d; ++k) {
            const uint32_t w = ordmap(pts[(size_t)k * n + id]);
            le &= w <= x[k];
            Kr += w;
        }
        pruned = le && Kr != K;   // all coordinates <= and not all equal (Def. 1)
    }
    if (!pruned) res[atomicAdd(kept, 1u)] = t;
}

// y[i] = -log1p(dc[i] * scale) / log1p(n) in float64, rounded once to float32;
// dc arrives in the same words as uint32.
__global__ void k_targets(uint32_t *__restrict__ y, uint32_t n, double scale, double norm,
                          const uint32_t *__restrict__ kept, uint32_t *__restrict__ kept_out)
{
    if (kept_out && blockIdx.x == 0 && threadIdx.x == 0) *kept_out = *kept;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double v = -log1p((double)y[i] * scale) / norm;
        y[i] = __float_as_uint((float)v);
    }
}

// ------------------------------------------------------------------ C-ABI
static int mlp_alloc(sky_mlp *M)
{
    const size_t pb = (size_t)M->np * 4;
    if (hipMalloc(&M->P, pb) != hipSuccess || hipMalloc(&M->m, pb) != hipSuccess ||
        hipMalloc(&M->v, pb) != hipSuccess || hipMalloc(&M->A1, 4 * 64 * sizeof(bf16x8)) != hipSuccess ||
        hipMalloc(&M->A2, 8 * 64 * sizeof(bf16x8)) != hipSuccess ||
        hipMalloc(&M->C1, 4 * 64 * sizeof(f32x4)) != hipSuccess ||
        hipMalloc(&M->C2, 4 * 64 * sizeof(f32x4)) != hipSuccess ||
        hipMalloc(&M->W3, 4 * 64 * sizeof(f32x4)) != hipSuccess || hipMalloc(&M->b3, 64) != hipSuccess ||
        hipMalloc(&M->grad, pb) != hipSuccess || hipMalloc(&M->loss, 64) != hipSuccess)
        return SKY_ERR_OOM;
    hipMemset(M->m, 0, pb);
    hipMemset(M->v, 0, pb);
    return SKY_OK;
}

static void mlp_free(sky_mlp *M)
{
    void *ps[] = {M->P, M->m, M->v, M->A1, M->A2, M->C1, M->C2, M->W3, M->b3, M->partial, M->grad, M->loss};
    for (void *p : ps)
        if (p) hipFree(p);
}

static int mlp_repack(sky_mlp *M, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(64), 0, s, M->P, M->d, M->A1, M->A2, M->C1, M->C2, M->W3, M->b3);
    return hipGetLastError() == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

// SplitMix64 (Steele, Lea, Flood 2014): a counter-based generator for the
// default initialisation.
static uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static double unif(uint64_t seed, uint64_t i) { return (double)(splitmix64(seed * 0x100000001B3ull + i) >> 11) * 0x1.0p-53; }

extern "C" int sky_mlp_create(sky_ctx *ctx, int32_t d, int32_t hidden, const float *init, uint64_t seed,
                              sky_mlp **out)
{
    if (!out) return SKY_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctx || d < 1 || d > SKY_MAXD || hidden != MLP_H) return SKY_ERR_INVALID_ARG;
    sky_mlp *M = new sky_mlp();
    M->serial = ++g_mlp_serial;
    M->device = sky_ctx_device(ctx);
    M->d = d;
    M->np = sky_mlp_nparams(d, hidden);
    if (hipSetDevice(M->device) != hipSuccess) { delete M; return SKY_ERR_HIP; }
    if (mlp_alloc(M) != SKY_OK) { mlp_free(M); delete M; return SKY_ERR_OOM; }
    const MlpLayout L{d, MLP_H};
    std::string host;
    float *h = new float[M->np];
    if (init) {
        memcpy(h, init, (size_t)M->np * 4);
    } else {
        // non-negative weights, biases centring the pre-activations for inputs in [0,1]
        for (int j = 0; j < MLP_H; ++j) {
            double rs = 0.0;
            for (int k = 0; k < d; ++k) {
                const double w = 2.0 * unif(seed, L.W1() + j * d + k) / d;
                h[L.W1() + j * d + k] = (float)w;
                rs += w;
            }
            h[L.b1() + j] = (float)(-0.5 * rs + 0.2 * (unif(seed, L.b1() + j) - 0.5));
        }
        for (int j = 0; j < MLP_H; ++j) {
            double rs = 0.0;
            for (int k = 0; k < MLP_H; ++k) {
                const double w = 2.0 * unif(seed, L.W2() + j * MLP_H + k) / MLP_H;
                h[L.W2() + j * MLP_H + k] = (float)w;
                rs += w;
            }
            h[L.b2() + j] = (float)(-0.1 * rs);
        }
        for (int j = 0; j < MLP_H; ++j) h[L.w3() + j] = (float)(2.0 * unif(seed, L.w3() + j) / MLP_H);
        h[L.b3()] = 0.0f;
    }
    const bool ok = hipMemcpy(M->P, h, (size_t)M->np * 4, hipMemcpyHostToDevice) == hipSuccess;
    delete[] h;
    if (!ok) { mlp_free(M); delete M; return SKY_ERR_HIP; }
    hipLaunchKernelGGL(k_project, dim3(8), dim3(256), 0, 0, M->P, d, M->np);
    if (mlp_repack(M, 0) != SKY_OK || hipDeviceSynchronize() != hipSuccess) { mlp_free(M); delete M; return SKY_ERR_HIP; }
    *out = M;
    return SKY_OK;
}

extern "C" void sky_mlp_destroy(sky_mlp *M)
{
    if (!M) return;
    hipSetDevice(M->device);
    mlp_free(M);
    delete M;
}

extern "C" int sky_mlp_get_params(const sky_mlp *M, float *host_out, int64_t cap)
{
    if (!M || !host_out || cap < M->np) return SKY_ERR_INVALID_ARG;
    hipSetDevice(M->device);
    return hipMemcpy(host_out, M->P, (size_t)M->np * 4, hipMemcpyDeviceToHost) == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

// File: "SKYMLP01", int32 d, int32 h, int64 nparams, int64 step, then float32
// master parameters, Adam first and second moments (little-endian).
extern "C" int sky_mlp_save(const sky_mlp *M, const char *path)
{
    if (!M || !path) return SKY_ERR_INVALID_ARG;
    hipSetDevice(M->device);
    const size_t nb = (size_t)M->np * 4;
    float *buf = new float[3 * M->np];
    bool ok = hipMemcpy(buf, M->P, nb, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(buf + M->np, M->m, nb, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(buf + 2 * M->np, M->v, nb, hipMemcpyDeviceToHost) == hipSuccess;
    FILE *f = ok ? fopen(path, "wb") : nullptr;
    if (f) {
        const char magic[8] = {'S', 'K', 'Y', 'M', 'L', 'P', '0', '1'};
        const int32_t dh[2] = {M->d, M->h};
        const int64_t ns[2] = {M->np, M->step};
        ok = fwrite(magic, 1, 8, f) == 8 && fwrite(dh, 4, 2, f) == 2 && fwrite(ns, 8, 2, f) == 2 &&
             fwrite(buf, 4, 3 * M->np, f) == (size_t)(3 * M->np);
        ok = (fclose(f) == 0) && ok;
    } else {
        ok = false;
    }
    delete[] buf;
    return ok ? SKY_OK : SKY_ERR_INVALID_ARG;
}

extern "C" int sky_mlp_load(sky_ctx *ctx, const char *path, sky_mlp **out)
{
    if (!ctx || !path || !out) return SKY_ERR_INVALID_ARG;
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return SKY_ERR_INVALID_ARG;
    char magic[8];
    int32_t dh[2];
    int64_t ns[2];
    if (fread(magic, 1, 8, f) != 8 || memcmp(magic, "SKYMLP01", 8) != 0 || fread(dh, 4, 2, f) != 2 ||
        fread(ns, 8, 2, f) != 2 || dh[0] < 1 || dh[0] > SKY_MAXD || dh[1] != MLP_H ||
        ns[0] != sky_mlp_nparams(dh[0], dh[1])) {
        fclose(f);
        return SKY_ERR_MODEL;
    }
    float *buf = new float[3 * ns[0]];
    const bool rd = fread(buf, 4, 3 * ns[0], f) == (size_t)(3 * ns[0]);
    fclose(f);
    if (!rd) { delete[] buf; return SKY_ERR_MODEL; }
    sky_mlp *M = nullptr;
    int rc = sky_mlp_create(ctx, dh[0], dh[1], buf, 0, &M);
    if (rc == SKY_OK) {
        const size_t nb = (size_t)M->np * 4;
        if (hipMemcpy(M->m, buf + M->np, nb, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(M->v, buf + 2 * M->np, nb, hipMemcpyHostToDevice) != hipSuccess)
            rc = SKY_ERR_HIP;
        M->step = ns[1];
    }
    delete[] buf;
    if (rc != SKY_OK) { sky_mlp_destroy(M); return rc; }
    *out = M;
    return SKY_OK;
}

extern "C" int sky_mlp_score(sky_ctx *ctx, const sky_mlp *M, const float *pts, int64_t n, int32_t d, float *out,
                             void *stream)
{
    if (!ctx || !M) return SKY_ERR_INVALID_ARG;
    if (n < 0 || n >= (1ll << 31) || (n > 0 && (!pts || !out))) return SKY_ERR_INVALID_ARG;
    if (d != M->d) return SKY_ERR_MODEL;
    hipSetDevice(M->device);
    hipStream_t s = (hipStream_t)stream;
    const int rc = sky_mlp_score_internal(M, pts, (uint32_t)n, d, out, s);
    if (rc != SKY_OK) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

static int ensure_partial(sky_mlp *M, int64_t nwg)
{
    if (nwg <= M->partial_cap) return SKY_OK;
    if (M->partial) hipFree(M->partial);
    M->partial = nullptr;
    M->partial_cap = 0;
    // one extra row per workgroup holds the loss partials
    if (hipMalloc(&M->partial, (size_t)nwg * (M->np + 1) * 4) != hipSuccess) return SKY_ERR_OOM;
    M->partial_cap = nwg;
    return SKY_OK;
}

static int loss_grad_async(sky_mlp *M, const float *pts, uint32_t n_stride, uint32_t first, uint32_t count, int d,
                           const float *y, float *grad, float *loss, hipStream_t s)
{
    const int64_t nch = (count + TR_P - 1) / TR_P;
    if (nch == 0) return SKY_OK;
    const int64_t nwg = nch < TR_MAXWG ? nch : TR_MAXWG;
    int rc = ensure_partial(M, nwg);
    if (rc != SKY_OK) return rc;
    float *loss_partial = M->partial + (size_t)nwg * M->np;
    const float inv_n = 1.0f / (float)count;
    if (d <= 8)
        hipLaunchKernelGGL(k_mlp_fwd_bwd<8>, dim3((unsigned)nwg), dim3(TR_P * TR_WAVES), 0, s, M->P, pts, n_stride,
                           first, count, d, y, inv_n, M->partial, M->np, loss_partial);
    else
        hipLaunchKernelGGL(k_mlp_fwd_bwd<16>, dim3((unsigned)nwg), dim3(TR_P * TR_WAVES), 0, s, M->P, pts, n_stride,
                           first, count, d, y, inv_n, M->partial, M->np, loss_partial);
    unsigned blocks = (unsigned)((M->np + 255) / 256);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks), dim3(256), 0, s, M->partial, (int)nwg, M->np, grad, loss_partial,
                       inv_n, loss);
    return hipGetLastError() == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

extern "C" int sky_mlp_loss_grad(sky_ctx *ctx, const sky_mlp *Mc, const float *pts, int64_t n, int32_t d,
                                 const float *y, float *grad, float *loss, void *stream)
{
    sky_mlp *M = const_cast<sky_mlp *>(Mc);
    if (!ctx || !M || n < 1 || n >= (1ll << 31) || !pts || !y || !grad || !loss) return SKY_ERR_INVALID_ARG;
    if (d != M->d) return SKY_ERR_MODEL;
    hipSetDevice(M->device);
    hipStream_t s = (hipStream_t)stream;
    const int rc = loss_grad_async(M, pts, (uint32_t)n, 0, (uint32_t)n, d, y, grad, loss, s);
    if (rc != SKY_OK) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

static int adam_async(sky_mlp *M, const float *grad, float lr, float b1, float b2, float eps, int64_t step,
                      hipStream_t s)
{
    const float c1 = (float)(1.0 - pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)step));
    unsigned blocks = (unsigned)((M->np + 255) / 256);
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks), dim3(256), 0, s, M->P, M->m, M->v, grad, M->d, M->np, lr, b1, b2, eps,
                       c1, c2);
    M->step = step;
    return mlp_repack(M, s);
}

extern "C" int sky_mlp_adam_step(sky_ctx *ctx, sky_mlp *M, const float *grad, float lr, float beta1, float beta2,
                                 float eps, int64_t step, void *stream)
{
    if (!ctx || !M || !grad || step < 1) return SKY_ERR_INVALID_ARG;
    hipSetDevice(M->device);
    hipStream_t s = (hipStream_t)stream;
    const int rc = adam_async(M, grad, lr, beta1, beta2, eps, step, s);
    if (rc != SKY_OK) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

extern "C" int sky_mlp_train(sky_ctx *ctx, sky_mlp *M, const float *pts, int64_t n, int32_t d, const float *y,
                             const sky_train_opts *to, float *loss_out, void *stream)
{
    if (!ctx || !M || !to || n < 1 || n >= (1ll << 31) || !pts || !y) return SKY_ERR_INVALID_ARG;
    if (d != M->d) return SKY_ERR_MODEL;
    if (to->epochs < 1 || to->batch < 1) return SKY_ERR_INVALID_ARG;
    hipSetDevice(M->device);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t nb = (uint32_t)((n + to->batch - 1) / to->batch);
    float *loss_hist = nullptr;
    if (hipMalloc(&loss_hist, (size_t)nb * 4) != hipSuccess) return SKY_ERR_OOM;
    int rc = SKY_OK;
    for (int e = 0; e < to->epochs && rc == SKY_OK; ++e) {
        for (uint32_t b = 0; b < nb && rc == SKY_OK; ++b) {
            const uint32_t first = b * (uint32_t)to->batch;
            const uint32_t cnt = (uint32_t)((int64_t)first + to->batch <= n ? to->batch : n - first);
            rc = loss_grad_async(M, pts, (uint32_t)n, first, cnt, d, y, M->grad, loss_hist + b, s);
            if (rc == SKY_OK) rc = adam_async(M, M->grad, to->lr, to->beta1, to->beta2, to->eps, M->step + 1, s);
        }
    }
    if (rc == SKY_OK && loss_out) {
        float *h = new float[nb];
        if (hipMemcpyAsync(h, loss_hist, (size_t)nb * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = SKY_ERR_HIP;
        double a = 0.0;
        for (uint32_t b = 0; b < nb; ++b) a += h[b];
        *loss_out = (float)(a / nb);
        delete[] h;
    }
    if (rc == SKY_OK && hipStreamSynchronize(s) != hipSuccess) rc = SKY_ERR_HIP;
    hipFree(loss_hist);
    return rc;
}

// Launch of the count kernel on stream s (n >= 1, 1 <= d <= 16); m_dev, when
// not NULL, holds the sample size on the device and overrides m.
static int domcount_launch(const float *pts, uint32_t n, int32_t d, const uint32_t *sample, uint32_t m,
                           const uint32_t *m_dev, int reverse, uint32_t *out, hipStream_t s)
{
    uint32_t blocks = (n + SKY_WG - 1) / SKY_WG;
    if (blocks > 4096) blocks = 4096;
    const int DP = sky_dp(d);
#define D_CASE(X)                                                                                                \
    case X:                                                                                                      \
        hipLaunchKernelGGL(k_domcount<X>, dim3(blocks), dim3(SKY_WG), 0, s, pts, n, d, sample, m, m_dev, reverse, \
                           out);                                                                                  \
        break;
    switch (DP) {
        D_CASE(4) D_CASE(8) D_CASE(12) D_CASE(16) D_CASE(20)
        default: return SKY_ERR_INVALID_ARG;
    }
#undef D_CASE
    return hipGetLastError() == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

static int domcount_impl(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *sample, int64_t m,
                         int reverse, uint32_t *out, void *stream)
{
    if (!ctx || d < 1 || d > SKY_MAXD || n < 0 || n >= (1ll << 31) || m < 0 || m >= (1ll << 31))
        return SKY_ERR_INVALID_ARG;
    if (n == 0) return SKY_OK;
    if (!pts || !out || (m > 0 && !sample)) return SKY_ERR_INVALID_ARG;
    hipSetDevice(sky_ctx_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const int rc = domcount_launch(pts, (uint32_t)n, d, sample, (uint32_t)m, nullptr, reverse, out, s);
    if (rc != SKY_OK) return rc;
    return hipStreamSynchronize(s) == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

extern "C" int sky_domcount(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *sample, int64_t m,
                            uint32_t *out, void *stream)
{
    return domcount_impl(ctx, pts, n, d, sample, m, 0, out, stream);
}

extern "C" int sky_mlp_targets(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *sample,
                               int64_t m, const uint32_t *reps, int64_t nreps, float *y, int64_t *kept_out,
                               void *stream)
{
    if (!ctx || d < 1 || d > SKY_MAXD || n < 0 || n >= (1ll << 31) || m < 0 || m >= (1ll << 31) || nreps < 0 ||
        nreps >= (1ll << 31))
        return SKY_ERR_INVALID_ARG;
    if (kept_out) *kept_out = 0;
    if (n == 0) return SKY_OK;
    if (!pts || !y || (m > 0 && !sample) || (nreps > 0 && !reps)) return SKY_ERR_INVALID_ARG;
    hipSetDevice(sky_ctx_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    uint32_t *res = nullptr;   // [0]: the count, then the residual ids
    if (hipMalloc(&res, ((size_t)m + 1) * 4) != hipSuccess) return SKY_ERR_OOM;
    int rc = SKY_OK;
    uint32_t kept = 0;
    if (hipMemsetAsync(res, 0, 4, s) != hipSuccess) rc = SKY_ERR_HIP;
    if (rc == SKY_OK && m > 0) {
        hipLaunchKernelGGL(k_residual, dim3((unsigned)((m + SKY_WG - 1) / SKY_WG)), dim3(SKY_WG), 0, s, pts,
                           (uint32_t)n, d, sample, (uint32_t)m, reps, (uint32_t)nreps, res + 1, res);
        if (hipGetLastError() != hipSuccess) rc = SKY_ERR_HIP;
    }
    if (rc == SKY_OK && (hipMemcpyAsync(&kept, res, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
        rc = SKY_ERR_HIP;
    // the counts land in y's words, then become the targets in place
    if (rc == SKY_OK) rc = domcount_impl(ctx, pts, n, d, res + 1, kept, 0, (uint32_t *)y, stream);
    if (rc == SKY_OK) {
        const double scale = m > 0 ? (double)n / (double)m : 0.0;
        unsigned blocks = (unsigned)((n + 255) / 256);
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_targets, dim3(blocks), dim3(256), 0, s, (uint32_t *)y, (uint32_t)n, scale,
                           log1p((double)n), res, nullptr);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = SKY_ERR_HIP;
    }
    hipFree(res);
    if (rc == SKY_OK && kept_out) *kept_out = kept;
    return rc;
}

// ------------------------------------------------------------------ allocation-free targets
// Scratch of sky_mlp_targets_noalloc: word 0 counts the residual sample, its
// ids start at word NA_IDS. Each device holds its own copy for the life of the
// process; host code reaches it only through the address looked up per device
// at context creation (the array's name is not a device address on the host).
#define NA_IDS 64u
static __device__ __align__(256) uint32_t scratch[NA_IDS + SKY_NOALLOC_MAX_M];
static uint32_t *g_scratch_dev[SKY_MAX_DEVICES];
static std::mutex g_scratch_mu;

int sky_noalloc_setup(int device)
{
    if (device < 0 || device >= SKY_MAX_DEVICES) return SKY_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return SKY_OK;
    void *p = nullptr;
    // the caller has made `device` current
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SKY_ERR_HIP;
    g_scratch_dev[device] = (uint32_t *)p;
    return SKY_OK;
}

__global__ void k_zero_word(uint32_t *w) { *w = 0u; }

extern "C" int sky_mlp_targets_noalloc(sky_ctx *ctx, const float *pts, int64_t n, int32_t d,
                                       const uint32_t *sample, int64_t m, const uint32_t *reps, int64_t nreps,
                                       float *y, uint32_t *kept_dev, void *stream)
{
    if (!ctx || d < 1 || d > SKY_MAXD || n < 0 || n >= (1ll << 31) || m < 0 || nreps < 0 || nreps >= (1ll << 31))
        return SKY_ERR_INVALID_ARG;
    if (m > (int64_t)SKY_NOALLOC_MAX_M) return SKY_ERR_CAPACITY;
    if (n == 0) return SKY_OK;
    if (!pts || !y || (m > 0 && !sample) || (nreps > 0 && !reps)) return SKY_ERR_INVALID_ARG;
    const int dev = sky_ctx_device(ctx);
    uint32_t *scr = dev >= 0 && dev < SKY_MAX_DEVICES ? g_scratch_dev[dev] : nullptr;
    if (!scr) return SKY_ERR_HIP;   // set up by sky_create on this device
    hipSetDevice(dev);
    hipStream_t s = (hipStream_t)stream;
    // the count starts at zero on every call (a kernel, not a memset: the call may be captured)
    hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, s, scr);
    if (m > 0)
        hipLaunchKernelGGL(k_residual, dim3((unsigned)((m + SKY_WG - 1) / SKY_WG)), dim3(SKY_WG), 0, s, pts,
                           (uint32_t)n, d, sample, (uint32_t)m, reps, (uint32_t)nreps, scr + NA_IDS, scr);
    if (hipGetLastError() != hipSuccess) return SKY_ERR_HIP;
    int rc = domcount_launch(pts, (uint32_t)n, d, scr + NA_IDS, 0u, scr, 0, (uint32_t *)y, s);
    if (rc != SKY_OK) return rc;
    const double scale = m > 0 ? (double)n / (double)m : 0.0;
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_targets, dim3(blocks), dim3(256), 0, s, (uint32_t *)y, (uint32_t)n, scale,
                       log1p((double)n), scr, kept_dev);
    return hipGetLastError() == hipSuccess ? SKY_OK : SKY_ERR_HIP;
}

extern "C" int sky_domby(sky_ctx *ctx, const float *pts, int64_t n, int32_t d, const uint32_t *by, int64_t m,
                         uint32_t *out, void *stream)
{
    return domcount_impl(ctx, pts, n, d, by, m, 1, out, stream);
}
