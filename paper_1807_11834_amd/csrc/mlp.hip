// mlp.hip -- the learned velocity surrogate on the gfx950 matrix cores.
//
// The surrogate predicts the sub-bulk part of the fluid velocity at a particle
// (fine-grid lookup minus bulk trilinear interpolation) from the 3x3x3 bulk
// stencil around its cell, its in-cell offset and its diameter.  All products
// are v_mfma_f32_16x16x32_bf16: BF16 operands (rounded to nearest even), FP32
// accumulation.
//
// Operand layout of one 16x16x32 product on a 64-lane wave (lane l, n = l % 16,
// g = l / 16): the A operand lane holds row n and eight contraction slots of
// group g, the B operand lane holds column n and the same eight slots, and the
// result lane holds column n, rows 4g .. 4g+3.  Which contraction index a slot
// stands for is a labelling shared by A and B: any permutation works as long as
// both operands use it.
//
// Products are written "transposed": weights are the A operand (rows = output
// neurons), activations the B operand (columns = particles).  The result of one
// layer (column = particle, rows = neurons 4g..4g+3 of a 16-row block) is then
// already the B operand of the next layer once two row blocks are paired into
// one 32-wide slot group: slots 0-3 <- rows 32q+4g+j, slots 4-7 <- rows
// 32q+16+4g+j.  The in-step inference kernel chains the four layers this way in
// registers, with the weights pre-permuted into that slot order in LDS.
//
// The training pass chains forward and backward the same way, a 16-row tile
// per pair of waves, and writes transposed copies of the layer inputs and
// output gradients for the weight-gradient products, whose contraction runs
// over the batch.  Batch inference on given features runs layer by layer over HBM in
// the natural slot order (rows k = 32q + 8g + i).  Every reduction has a fixed
// order.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "mlp.hpp"
#include "sample.hpp"

namespace cpl {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((__vector_size__(16)));
typedef float f32x4 __attribute__((__vector_size__(16)));

// float -> bfloat16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ uint32_t bf16_bits(float x) { return pack2(x, 0.f) & 0xffffu; }
__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ bf16x8 load8(const uint16_t *p) { return as_bf16x8(*reinterpret_cast<const uint4 *>(p)); }
__device__ __forceinline__ bf16x8 zero8() { return as_bf16x8(make_uint4(0u, 0u, 0u, 0u)); }
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// tanh-form GELU 0.5 z (1 + tanh(u)), u = sqrt(2/pi) (z + 0.044715 z^3), written
// as z * sigma(2u) with sigma(2u) = 1 / (1 + 2^(-2u log2 e)): one exp2 and one
// reciprocal (hardware, ~1 ulp).  For z -> -inf, 2^(...) -> inf and the result
// -> -0; for z -> +inf it -> z.  Derivative: with s = sigma(2u),
//   gelu'(z) = s + 2 z s (1 - s) du/dz,  du/dz = sqrt(2/pi) (1 + 3 * 0.044715 z^2).
constexpr float kGc = 0.7978845608028654f, kGa = 0.044715f;
constexpr float kGk = 2.3022081983914574f;   // 2 sqrt(2/pi) log2(e)
__device__ __forceinline__ float sig2u(float z) {
    const float t = fmaf(-kGk * kGa, z * z, -kGk);   // -2u log2(e) / z
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(z * t));
}
__device__ __forceinline__ float gelu(float z) { return z * sig2u(z); }
__device__ __forceinline__ float gelu_grad(float z) {
    const float s = sig2u(z);
    return s + 2.f * z * s * (1.f - s) * (kGc * fmaf(3.f * kGa, z * z, 1.f));
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// ---------------------------------------------------------------------------
// Parameter bookkeeping
// ---------------------------------------------------------------------------
// Flat parameter index -> (layer, is_weight, k, m).
__device__ __forceinline__ void decode_param(int64_t i, int &l, bool &w, int &k, int &m) {
    constexpr int64_t kW1 = off_w(1), kW2 = off_w(2), kW3 = off_w(3);
    constexpr int64_t kB0 = off_b(0), kB1 = off_b(1), kB2 = off_b(2), kB3 = off_b(3);
    l = i < kW1 ? 0 : (i < kW2 ? 1 : (i < kW3 ? 2 : 3));
    const int64_t w0 = l == 0 ? 0 : (l == 1 ? kW1 : (l == 2 ? kW2 : kW3));
    const int64_t b0 = l == 0 ? kB0 : (l == 1 ? kB1 : (l == 2 ? kB2 : kB3));
    const int fo = l == 3 ? kOut : kHid;
    w = i < b0;
    if (w) {
        k = (int)((i - w0) / fo);
        m = (int)((i - w0) % fo);
    } else {
        k = 0;
        m = (int)(i - b0);
    }
}

struct WPtrs {
    uint16_t *wt[4], *wn[4], *wtp[4], *wnp[4];
};

__device__ __forceinline__ void write_bf16_copies(const WPtrs &w, int l, int k, int m, float p) {
    const uint16_t b = (uint16_t)bf16_bits(p);
    w.wt[l][(int64_t)m * kpad(l) + k] = b;
    if (l > 0) {
        w.wn[l][(int64_t)k * cpad(l) + m] = b;
        w.wtp[l][(int64_t)m * kpad(l) + perm_col(k)] = b;
        w.wnp[l][(int64_t)k * cpad(l) + perm_col(m)] = b;
    }
}

__global__ __launch_bounds__(kBlock) void k_cast(const float *__restrict__ params, WPtrs w) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= kNParam) return;
    int l, k, m;
    bool isw;
    decode_param(i, l, isw, k, m);
    if (isw) write_bf16_copies(w, l, k, m, params[i]);
}

// Adam (bias-corrected) on the FP32 master parameters, then the BF16 copies.
__global__ __launch_bounds__(kBlock) void k_adam(const float *__restrict__ grads, float *__restrict__ params,
                                                 float *__restrict__ mom1, float *__restrict__ mom2, WPtrs w,
                                                 float lr, float b1, float omb1, float b2, float omb2, float eps,
                                                 float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= kNParam) return;
    const float g = grads[i];
    const float m = b1 * mom1[i] + omb1 * g;
    const float v = b2 * mom2[i] + omb2 * g * g;
    const float p = params[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    mom1[i] = m;
    mom2[i] = v;
    params[i] = p;
    int l, k, mm;
    bool isw;
    decode_param(i, l, isw, k, mm);
    if (isw) write_bf16_copies(w, l, k, mm, p);
}

// ---------------------------------------------------------------------------
// Batch inference on given features
// ---------------------------------------------------------------------------
// X0[b][k] = bf16((feat[b][k] - mean[k]) / std[k]) for k < 193, 0 up to 224.
// A workgroup takes 64 rows: their features are read row by row (consecutive
// threads, consecutive features) and standardised into an LDS tile, from which
// the rows leave as 16-byte stores.
constexpr int kStdRows = 64;
constexpr int kStdPitch = kK1 + 2;   // BF16 elements per LDS row
__global__ __launch_bounds__(kBlock) void k_standardise(const float *__restrict__ feat, int64_t B,
                                                        const float *__restrict__ mean_inv, uint16_t *__restrict__ x0) {
    __shared__ uint16_t tile[kStdRows * kStdPitch];
    const int64_t b0 = (int64_t)blockIdx.x * kStdRows;
    const int nr = (int)(B - b0 < kStdRows ? B - b0 : kStdRows);
    for (int e = threadIdx.x; e < nr * kK1; e += kBlock) {
        const int r = e / kK1, k = e % kK1;
        float v = 0.f;
        if (k < kFeat) v = (feat[(b0 + r) * kFeat + k] - mean_inv[k]) * mean_inv[kK1 + k];
        tile[r * kStdPitch + k] = (uint16_t)bf16_bits(v);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * (kK1 / 8); e += kBlock) {
        const int r = e / (kK1 / 8), k0 = 8 * (e % (kK1 / 8));
        const uint16_t *t = tile + r * kStdPitch + k0;
        const uint4 pk = make_uint4(t[0] | ((uint32_t)t[1] << 16), t[2] | ((uint32_t)t[3] << 16),
                                    t[4] | ((uint32_t)t[5] << 16), t[6] | ((uint32_t)t[7] << 16));
        *reinterpret_cast<uint4 *>(x0 + (b0 + r) * kK1 + k0) = pk;
    }
}

// One dense layer of the batch forward pass for 16-row tiles, one wave per tile:
//   Z = X W + b (X [B][32 KB] BF16, W^T [16 MB][32 KB] BF16), then
//   hidden: gelu(Z) -> H (BF16 [B][16 MB]); output (MB = 1): Z -> Y [B][16].
template <int KB, int MB, bool OUT>
__global__ __launch_bounds__(kBlock) void k_dense(const uint16_t *__restrict__ X, const uint16_t *__restrict__ WT,
                                                  const float *__restrict__ bias, int M, int64_t B,
                                                  float *__restrict__ Y, uint16_t *__restrict__ H) {
    constexpr int KP = 32 * KB, MP = 16 * MB;
    const int lane = lane_id(), n = lane & 15, g = lane >> 4;
    const int64_t ntile = (B + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (tile >= ntile) return;   // whole wave
    const int64_t b = tile * 16 + n;
    const bool valid = b < B;
    bf16x8 xb[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) xb[kb] = valid ? load8(X + b * KP + 32 * kb + 8 * g) : zero8();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) acc = mma(load8(WT + (int64_t)(16 * mb + n) * KP + 32 * kb + 8 * g), xb[kb], acc);
        const int m0 = 16 * mb + 4 * g;
        float z[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) z[j] = acc[j] + ((m0 + j < M) ? bias[m0 + j] : 0.f);
        if (!valid) continue;
        if constexpr (OUT) {
            *reinterpret_cast<float4 *>(Y + b * MP + m0) = make_float4(z[0], z[1], z[2], z[3]);
        } else {
            *reinterpret_cast<uint2 *>(H + b * MP + m0) =
                make_uint2(pack2(gelu(z[0]), gelu(z[1])), pack2(gelu(z[2]), gelu(z[3])));
        }
    }
}

// ---------------------------------------------------------------------------
// Training pass: standardisation, forward, loss and backward of 32 rows by a
// workgroup of four waves
// ---------------------------------------------------------------------------
// Batch rows are the product columns (lane n holds row 16 t + n of tile t) and
// neurons the product rows, as in the in-step inference.  A layer's result is
// the next B operand in the permuted slot order (slots 4s + j of group g <-
// neuron 32q + 16s + 4g + j); the weight fragments are read in the same order
// from the permuted copies, and the backward products take the output
// gradients in the same layout.  The four waves of a workgroup split every
// 128-neuron layer: wave w computes neuron blocks 2w and 2w + 1 (one
// contraction block q = w of the next product) for both 16-row tiles, so that
// each weight fragment it loads feeds two products, and keeps their gelu'(Z),
// formed in the forward pass with gelu (one exponential).  The other three
// contraction blocks of the next B operand are read back from the LDS stage
// below after a workgroup barrier; so is the layer-1 input, of which each wave
// loads and standardises two of the seven 32-feature blocks.  With an 80 KB
// stage and at most 256 registers per wave, two workgroups share a compute
// unit.
//
// For the weight-gradient products over the batch the pass writes the BF16
// layer inputs and the BF16 output gradients transposed, as the rows of one
// 1008-row matrix (x0 224, h 3 x 128, dZ 3 x 128 + 16) in blocks of 32 batch
// rows.  These are staged in LDS, [row][32 batch rows of the workgroup], and
// leave at the end as the workgroup's contiguous block: a wave's stores and
// loads share one in-order completion counter, so a store issued between the
// weight loads of two layers would make the second layer wait for it.  The
// bias gradients are the column sums of the FP32 output gradients: summed in
// FP64 over the 16 rows of a tile (a fixed butterfly), then over the two tiles
// of a workgroup in tile order, into part_b[l][workgroup][MP].  The loss
// partial of a tile is sum 0.5 (y - t)^2 / B.  B is a multiple of 32: every
// workgroup has both tiles.
constexpr int kTrainTiles = 2;                    // 16-row tiles per workgroup
static_assert(kTrainGroupRows == 16 * kTrainTiles, "two 16-row tiles per workgroup");
constexpr int kTrainWaves = 4;                    // a quarter of every layer's neurons each
constexpr int kTrainThreads = kTrainWaves * kWave;
constexpr int kBiasCols = 3 * kHid + 16;          // bias-gradient columns, layers 1-4
// Staged transposed rows: layer-1 input (224), hidden activations (3 x 128),
// output gradients (3 x 128 + 16).  36 BF16 per staged row: the four rows that
// one access instruction touches per lane group (4 apart) then fall 8 banks
// apart.
constexpr int kStagePitch = kTrainGroupRows + 4;
constexpr int kStageHt = kTrHt, kStageDz = kTrDz, kStageRows = kTrRows;
static_assert(kStageRows % 16 == 0, "the output pass takes whole rows");

struct TrainArgs {
    const float *feat, *resid;
    const int32_t *idx;
    int64_t nrows, B;
    const float *mean_inv;
    float is[3], inv_b;
    const float *params;
    const uint16_t *wt0;              // layer-1 W^T, natural order
    const uint16_t *wtp[4], *wnp[4];  // layers 2-4, permuted order
    uint16_t *tr;   // transposed rows, blocks of kTrBlock batch rows
    double *part_b[4];
    double *loss_part;
};

// Four BF16 values (two packed words) of column col staged to rows r0 .. r0+3.
__device__ __forceinline__ void stage_t4(uint16_t *S, int r0, int col, uint32_t w0, uint32_t w1) {
    S[r0 * kStagePitch + col] = (uint16_t)(w0 & 0xffffu);
    S[(r0 + 1) * kStagePitch + col] = (uint16_t)(w0 >> 16);
    S[(r0 + 2) * kStagePitch + col] = (uint16_t)(w1 & 0xffffu);
    S[(r0 + 3) * kStagePitch + col] = (uint16_t)(w1 >> 16);
}
// The same four values read back as two packed words.
__device__ __forceinline__ void unstage_t4(const uint16_t *S, int r0, int col, uint32_t &w0, uint32_t &w1) {
    w0 = (uint32_t)S[r0 * kStagePitch + col] | ((uint32_t)S[(r0 + 1) * kStagePitch + col] << 16);
    w1 = (uint32_t)S[(r0 + 2) * kStagePitch + col] | ((uint32_t)S[(r0 + 3) * kStagePitch + col] << 16);
}

// Sum over the 16 lanes of a lane group (lanes with equal g), FP64.
__device__ __forceinline__ double sum16(double v) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Column sums over the 16 lanes of a lane group of the 8 values v = 4 b + j of
// a lane (FP32 in, FP64 sums): a reduce-scatter butterfly over lane bits 3, 2,
// 1 (each stage keeps half of the values, the upper half where the lane bit is
// set, adds the partner's copy of that half and sends the other half), then
// lanes n and n ^ 1 add their partial sums: both hold the sum of value n / 2.
// The adding order of every column is a fixed tree (a + b = b + a exactly, so
// partners agree).
__device__ __forceinline__ double colsum8(const float (&v)[8], int n) {
    double s4[4];
    const bool u3 = (n & 8) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float recv = __shfl_xor(u3 ? v[i] : v[i + 4], 8, kWave);
        s4[i] = (double)(u3 ? v[i + 4] : v[i]) + (double)recv;
    }
    double s2[2];
    const bool u2 = (n & 4) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) s2[i] = (u2 ? s4[i + 2] : s4[i]) + __shfl_xor(u2 ? s4[i] : s4[i + 2], 4, kWave);
    const bool u1 = (n & 2) != 0;
    const double s1 = (u1 ? s2[1] : s2[0]) + __shfl_xor(u1 ? s2[0] : s2[1], 2, kWave);
    return s1 + __shfl_xor(s1, 1, kWave);
}

// A quarter of a layer's output gradient (FP32, result layout; tiles t, blocks
// 2w + b): the BF16 values staged transposed (S, columns 16 t + n) and kept as
// packed words, the bias column sums of each tile into
// bs[t][16 (2w + b) + 4 g + j].
__device__ __forceinline__ void emit_grad(const f32x4 (&d)[2][2], int w, int n, int g, uint16_t *S,
                                          double (*bs)[kBiasCols], int bcol, uint32_t (&wv)[2][2][2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        float v[8];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            wv[t][b][0] = pack2(d[t][b][0], d[t][b][1]);
            wv[t][b][1] = pack2(d[t][b][2], d[t][b][3]);
            stage_t4(S, 16 * (2 * w + b) + 4 * g, 16 * t + n, wv[t][b][0], wv[t][b][1]);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[4 * b + j] = d[t][b][j];
        }
        const double cs = colsum8(v, n);   // value n / 2: block n / 8, row (n / 2) % 4
        if ((n & 1) == 0) bs[t][bcol + 16 * (2 * w + (n >> 3)) + 4 * g + ((n >> 1) & 3)] = cs;
    }
}

// A quarter of a hidden layer's result (tiles t, blocks 2w + b): Z = acc + b
// (bv: the bias values of the lane's rows), H = gelu(Z) as BF16 (staged
// transposed and kept as packed words), gelu'(Z) kept.
__device__ __forceinline__ void finish_hidden(const f32x4 (&acc)[2][2], const float4 (&bv)[2], int w, int n, int g,
                                              uint16_t *S, f32x4 (&gp)[2][2], uint32_t (&wv)[2][2][2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            float hv[4];
            const float bj[4] = {bv[b].x, bv[b].y, bv[b].z, bv[b].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float z = acc[t][b][j] + bj[j];
                const float s = sig2u(z);
                hv[j] = z * s;   // gelu(z)
                gp[t][b][j] = s + 2.f * z * s * (1.f - s) * (kGc * fmaf(3.f * kGa, z * z, 1.f));   // gelu'(z)
            }
            wv[t][b][0] = pack2(hv[0], hv[1]);
            wv[t][b][1] = pack2(hv[2], hv[3]);
            stage_t4(S, 16 * (2 * w + b) + 4 * g, 16 * t + n, wv[t][b][0], wv[t][b][1]);
        }
}

// The full B operands (four contraction blocks, both tiles) of a 128-neuron
// result split over the four waves: block q = w from the wave's own packed
// words, the others read back from their staged rows (S).
__device__ __forceinline__ void gather_operand(const uint32_t (&wv)[2][2][2], const uint16_t *S, int w, int n, int g,
                                               bf16x8 (&x)[2][4]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t p[4];
            if (q == w) {
                p[0] = wv[t][0][0];
                p[1] = wv[t][0][1];
                p[2] = wv[t][1][0];
                p[3] = wv[t][1][1];
            } else {
                unstage_t4(S, 16 * (2 * q) + 4 * g, 16 * t + n, p[0], p[1]);
                unstage_t4(S, 16 * (2 * q + 1) + 4 * g, 16 * t + n, p[2], p[3]);
            }
            x[t][q] = as_bf16x8(make_uint4(p[0], p[1], p[2], p[3]));
        }
}

// A quarter of a 128 x 128 product in the permuted order: f[b][q] = row
// 16 (2w + b) + n of Mp (a permuted copy, pitch P), contraction block q, one
// 16-byte load.  A layer's fragments are loaded as one batch, ahead of the
// work before the product, so that their latency overlaps it; the product
// then runs on registers, each fragment feeding both tiles.
template <int P>
__device__ __forceinline__ void load_frags(const uint16_t *__restrict__ Mp, int w, int n, int g, bf16x8 (&f)[2][4]) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) f[b][q] = load8(Mp + (16 * (2 * w + b) + n) * P + 32 * q + 8 * g);
}
// The bias values of a hidden layer for the lane's rows of blocks 2w, 2w + 1.
__device__ __forceinline__ void load_bias(const float *__restrict__ bias, int w, int g, float4 (&bv)[2]) {
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const float4 *>(bias + 16 * (2 * w + b) + 4 * g);
}
__device__ __forceinline__ void product(const bf16x8 (&f)[2][4], const bf16x8 (&x)[2][4], f32x4 (&acc)[2][2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc[t][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[t][b] = mma(f[b][q], x[t][q], acc[t][b]);
        }
}
// Keeps the loads above it from sinking towards their first use.
__device__ __forceinline__ void issue_fence() { __builtin_amdgcn_sched_barrier(0); }

__global__ __launch_bounds__(kTrainThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_train_tile(TrainArgs a) {
    __shared__ __align__(16) uint16_t stage[kStageRows * kStagePitch];
    __shared__ float norm[2 * kK1];
    __shared__ double bsum[kTrainTiles][kBiasCols];
    for (int i = threadIdx.x; i < 2 * kK1; i += kTrainThreads) norm[i] = a.mean_inv[i];
    __syncthreads();
    constexpr int64_t kOffB0 = off_b(0), kOffB1 = off_b(1), kOffB2 = off_b(2), kOffB3 = off_b(3);
    const int lane = lane_id(), n = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int64_t tile0 = (int64_t)blockIdx.x * kTrainTiles;
    uint16_t *sh = stage + kStageHt * kStagePitch, *sd = stage + kStageDz * kStagePitch;
    f32x4 acc[2][2], gp[3][2][2];
    uint32_t wv[2][2][2];
    bf16x8 x[2][4], f[2][4];
    float4 bv[2];

    // the rows of both tiles; this wave's share of the layer-1 input, feature
    // blocks kb = 2w, 2w + 1 (< 7), standardised and staged; the layer-1
    // weight fragments of its neuron blocks
    float t[2][4];
    {
        float fv[2][2][8];
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int64_t b = (tile0 + tt) * 16 + n;
            int64_t row = a.idx ? (int64_t)a.idx[b] : b;
            if (row < 0 || row >= a.nrows) row = 0;   // documented: indices must be in range; keeps loads in bounds
            const float *fr = a.feat + row * kFeat;
#pragma unroll
            for (int j = 0; j < 4; ++j) t[tt][j] = (g == 0 && j < kOut) ? a.resid[row * 3 + j] * a.is[j] : 0.f;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = 32 * (2 * w + kk) + 8 * g + i;
                    fv[tt][kk][i] = k < kFeat ? fr[k] : 0.f;
                }
        }
        bf16x8 f1[2][7];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int kb = 0; kb < 7; ++kb) f1[b][kb] = load8(a.wt0 + (16 * (2 * w + b) + n) * kK1 + 32 * kb + 8 * g);
        issue_fence();
#pragma unroll
        for (int tt = 0; tt < 2; ++tt)
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int kb = 2 * w + kk;
                if (kb < 7) {
                    float v[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int k = 32 * kb + 8 * g + i;
                        v[i] = k < kFeat ? (fv[tt][kk][i] - norm[k]) * norm[kK1 + k] : 0.f;
                    }
                    stage_t4(stage, 32 * kb + 8 * g, 16 * tt + n, pack2(v[0], v[1]), pack2(v[2], v[3]));
                    stage_t4(stage, 32 * kb + 8 * g + 4, 16 * tt + n, pack2(v[4], v[5]), pack2(v[6], v[7]));
                }
            }
        __syncthreads();   // the layer-1 input staged
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            bf16x8 xb[7];
#pragma unroll
            for (int kb = 0; kb < 7; ++kb) {
                uint32_t p[4];
                unstage_t4(stage, 32 * kb + 8 * g, 16 * tt + n, p[0], p[1]);
                unstage_t4(stage, 32 * kb + 8 * g + 4, 16 * tt + n, p[2], p[3]);
                xb[kb] = as_bf16x8(make_uint4(p[0], p[1], p[2], p[3]));
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc[tt][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 7; ++kb) acc[tt][b] = mma(f1[b][kb], xb[kb], acc[tt][b]);
            }
        }
    }
    load_frags<kHid>(a.wtp[1], w, n, g, f);
    load_bias(a.params + kOffB0, w, g, bv);
    issue_fence();
    finish_hidden(acc, bv, w, n, g, sh, gp[0], wv);
    __syncthreads();   // layer 1 staged
    gather_operand(wv, sh, w, n, g, x);
    product(f, x, acc);
    load_frags<kHid>(a.wtp[2], w, n, g, f);
    load_bias(a.params + kOffB1, w, g, bv);
    issue_fence();
    finish_hidden(acc, bv, w, n, g, sh + kHid * kStagePitch, gp[1], wv);
    __syncthreads();   // layer 2 staged
    gather_operand(wv, sh + kHid * kStagePitch, w, n, g, x);
    product(f, x, acc);
    bf16x8 fo[4], f4[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) fo[q] = load8(a.wtp[3] + n * kHid + 32 * q + 8 * g);
#pragma unroll
    for (int b = 0; b < 2; ++b) f4[b] = load8(a.wnp[3] + (16 * (2 * w + b) + n) * 32 + 8 * g);
    load_bias(a.params + kOffB2, w, g, bv);
    float yb[4] = {0.f, 0.f, 0.f, 0.f};   // output bias of the lane's rows m = 4 g + j
    if (g == 0)
#pragma unroll
        for (int j = 0; j < kOut; ++j) yb[j] = a.params[kOffB3 + j];
    issue_fence();
    finish_hidden(acc, bv, w, n, g, sh + 2 * kHid * kStagePitch, gp[2], wv);
    __syncthreads();   // layer 3 staged
    gather_operand(wv, sh + 2 * kHid * kStagePitch, w, n, g, x);

    // output layer (rows m = 4 g + j, three of them real) in every wave; the
    // loss, dY's staged rows and its bias sums from wave 0
    double lp[2];
    bf16x8 dy[2];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q) y = mma(fo[q], x[tt][q], y);
        float d[4];
        lp[tt] = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 4 * g + j;
            const float dd = m < kOut ? (y[j] + yb[j]) - t[tt][j] : 0.f;
            lp[tt] += 0.5 * (double)dd * (double)dd;
            d[j] = dd * a.inv_b;
        }
        const uint32_t w0 = pack2(d[0], d[1]), w1 = pack2(d[2], d[3]);
        dy[tt] = as_bf16x8(make_uint4(w0, w1, 0u, 0u));
        if (w == 0) {
            stage_t4(sd + 3 * kHid * kStagePitch, 4 * g, 16 * tt + n, w0, w1);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double s = sum16((double)d[j]);
                if (n == 0) bsum[tt][3 * kHid + 4 * g + j] = s;
            }
        }
    }
    // backward: dZ_l = (dZ_{l+1} W_{l+1}^T) .* gelu'(Z_l), l = 3, 2, 1
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc[tt][b] = mma(f4[b], dy[tt], f32x4{0.f, 0.f, 0.f, 0.f});
            acc[tt][b] *= gp[2][tt][b];
        }
    load_frags<kHid>(a.wnp[2], w, n, g, f);
    issue_fence();
    emit_grad(acc, w, n, g, sd + 2 * kHid * kStagePitch, bsum, 2 * kHid, wv);
    __syncthreads();   // dZ3 staged
    gather_operand(wv, sd + 2 * kHid * kStagePitch, w, n, g, x);
    product(f, x, acc);
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[tt][b] *= gp[1][tt][b];
    load_frags<kHid>(a.wnp[1], w, n, g, f);
    issue_fence();
    emit_grad(acc, w, n, g, sd + kHid * kStagePitch, bsum, kHid, wv);
    __syncthreads();   // dZ2 staged
    gather_operand(wv, sd + kHid * kStagePitch, w, n, g, x);
    product(f, x, acc);
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[tt][b] *= gp[0][tt][b];
    emit_grad(acc, w, n, g, sd, bsum, 0, wv);
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const double l = wave_sum(lp[tt]);
        if (lane == 0 && w == 0) a.loss_part[tile0 + tt] = l * (double)a.inv_b;
    }
    __syncthreads();   // the group is staged
    for (int c = threadIdx.x; c < kBiasCols; c += kTrainThreads) {
        const double sb = bsum[0][c] + bsum[1][c];
        const int l = c < 3 * kHid ? c / kHid : 3, m = c - l * kHid, MP = mpad(l);
        a.part_b[l][(int64_t)blockIdx.x * MP + m] = sb;
    }
    // the staged block out: kTrRows rows of 32 batch rows, 8 threads per row
    // with 4 batch rows (8 bytes) each
    uint16_t *dst = a.tr + (int64_t)blockIdx.x * kStageRows * kTrBlock;
    constexpr int kChunks = kStageRows * kTrBlock / 4, kU = 8;
    constexpr int kIter = (kChunks + kTrainThreads - 1) / kTrainThreads;
    for (int i0 = 0; i0 < kIter; i0 += kU) {
        uint2 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = threadIdx.x + kTrainThreads * (i0 + u);
            if (e < kChunks) v[u] = *reinterpret_cast<const uint2 *>(stage + (e >> 3) * kStagePitch + 4 * (e & 7));
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int e = threadIdx.x + kTrainThreads * (i0 + u);
            if (e < kChunks) *reinterpret_cast<uint2 *>(dst + 4 * e) = v[u];
        }
    }
}

// Weight gradients of one layer over a chunk of rows:
//   part_w[c][m][k] = sum_{b in chunk} dZ[b][m] H[b][k]   (BF16 x BF16, FP32 accumulate)
// from the training pass's transposed rows (dZ rows dz_row + 16 MT, H rows
// h_row + 16 KT, blocks of kTrBlock batch rows).  Rows in chunks of kChunk; B
// is a multiple of 32.  Each of the kWgradWaves waves of a workgroup owns
// output column blocks kt and keeps all MT row blocks in registers: per 32 rows
// it loads one H fragment and the MT dZ fragments and issues MT independent
// products.
constexpr int kWgradWaves = 8;
template <int MT, int KT>
__device__ __forceinline__ void wgrad_chunk(const uint16_t *__restrict__ tr, int dz_row, int h_row, int64_t B,
                                            float *__restrict__ part_w) {
    constexpr int MP = 16 * MT, KP = 16 * KT;
    constexpr int64_t kBlk = (int64_t)kTrRows * kTrBlock;   // elements per block of batch rows
    static_assert(kTrBlock == 32, "one block per 32-row product");
    const int lane = lane_id(), n = lane & 15, g = lane >> 4, wave = threadIdx.x >> 6;
    const int64_t c = blockIdx.x;
    const int64_t b0 = c * kChunk, b1 = (b0 + kChunk < B) ? b0 + kChunk : B;
    for (int kt = wave; kt < KT; kt += kWgradWaves) {
        f32x4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        const uint16_t *pb = tr + (int64_t)(h_row + 16 * kt + n) * kTrBlock + 8 * g;
        const uint16_t *pa = tr + (int64_t)(dz_row + n) * kTrBlock + 8 * g;
        // kU groups of 32 rows per round, all their loads issued before the
        // products (the rows are still summed in order)
        constexpr int kU = MT > 4 ? 4 : 8;
        for (int64_t bb = b0; bb < b1; bb += 32 * kU) {
            bf16x8 bv[kU];
            bf16x8 av[kU][MT];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t r = bb + 32 * u < b1 ? bb + 32 * u : b1 - 32;
                const int64_t o = (r / kTrBlock) * kBlk;
                bv[u] = load8(pb + o);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) av[u][mt] = load8(pa + 16 * mt * kTrBlock + o);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (bb + 32 * u >= b1) break;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = mma(av[u][mt], bv[u], acc[mt]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            float *o = part_w + (c * MP + 16 * mt + 4 * g) * KP + 16 * kt + n;
#pragma unroll
            for (int j = 0; j < 4; ++j) o[(int64_t)j * KP] = acc[mt][j];
        }
    }
}

// The four layers' weight gradients in one launch (blockIdx.y = layer), so
// that the short layers fill the tail of the long one.
struct WgradParts {
    float *w[4];
};
__global__ __launch_bounds__(kWgradWaves * kWave) void k_wgrad(const uint16_t *__restrict__ tr, int64_t B,
                                                               WgradParts parts) {
    switch (blockIdx.y) {
    case 0: wgrad_chunk<8, 14>(tr, kTrDz, 0, B, parts.w[0]); break;
    case 1: wgrad_chunk<8, 8>(tr, kTrDz + kHid, kTrHt, B, parts.w[1]); break;
    case 2: wgrad_chunk<8, 8>(tr, kTrDz + 2 * kHid, kTrHt + kHid, B, parts.w[2]); break;
    default: wgrad_chunk<1, 8>(tr, kTrDz + 3 * kHid, kTrHt + 2 * kHid, B, parts.w[3]); break;
    }
}

struct GradParts {
    const float *w[4];
    const double *b[4];
};

// Flat gradient vector from the partials.  Weight entries follow the
// partials' layout (per layer the padded [m][k] slots, k fastest), so that the
// loads of a wave are contiguous; each is summed by kRedGroups threads over
// interleaved chunks (c mod kRedGroups, two partial sums each) whose results
// are combined in a fixed order.  The bias entries are summed over the
// nchunk_b workgroup partials of the training pass (below).
constexpr int kRedGroups = 8;
constexpr int kRedEntries = kBlock / kRedGroups;   // entries per workgroup
constexpr int64_t kRedW1 = (int64_t)mpad(0) * kpad(0), kRedW2 = kRedW1 + (int64_t)mpad(1) * kpad(1),
                  kRedW3 = kRedW2 + (int64_t)mpad(2) * kpad(2), kRedTotal = kRedW3 + (int64_t)mpad(3) * kpad(3);
constexpr int kRedBias = 3 * kHid + kOut;          // bias entries (real ones)

__global__ __launch_bounds__(kBlock) void k_reduce_w(GradParts parts, int64_t nchunk, float *__restrict__ grads) {
    constexpr int64_t kOffW[4] = {off_w(0), off_w(1), off_w(2), off_w(3)};
    __shared__ double red[kRedGroups][kRedEntries];
    const int le = threadIdx.x % kRedEntries, grp = threadIdx.x / kRedEntries;
    const int64_t e = (int64_t)blockIdx.x * kRedEntries + le;
    const int l = e < kRedW1 ? 0 : (e < kRedW2 ? 1 : (e < kRedW3 ? 2 : 3));
    const int64_t r = e - (l == 0 ? 0 : (l == 1 ? kRedW1 : (l == 2 ? kRedW2 : kRedW3)));
    const int MP = l == 3 ? mpad(3) : kHid, KP = l == 0 ? kpad(0) : kHid;
    const int m = (int)(r / KP), k = (int)(r % KP);
    double s0 = 0.0, s1 = 0.0;
    if (e < kRedTotal) {
        const float *w = parts.w[l] + r;
        const int64_t stride = (int64_t)MP * KP;
        int64_t c = grp;
        for (; c + kRedGroups < nchunk; c += 2 * kRedGroups) {
            s0 += (double)w[c * stride];
            s1 += (double)w[(c + kRedGroups) * stride];
        }
        if (c < nchunk) s0 += (double)w[c * stride];
    }
    red[grp][le] = s0 + s1;
    __syncthreads();
    if (grp == 0 && e < kRedTotal) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kRedGroups; ++q) t += red[q][le];
        const int fi = l == 0 ? kFeat : kHid, fo = l == 3 ? kOut : kHid;
        if (k < fi && m < fo) grads[kOffW[l] + (int64_t)k * fo + m] = (float)t;
    }
}

// kRedBEntries consecutive bias entries per workgroup, kRedBLanes threads per
// entry over interleaved partials (c mod kRedBLanes; a wave reads 8 partials
// of 8 consecutive entries), then one thread per entry adds the lanes' sums
// in lane order.
constexpr int kRedBEntries = 8, kRedBLanes = 128, kRedBThreads = kRedBEntries * kRedBLanes;
__global__ __launch_bounds__(kRedBThreads) void k_reduce_b(GradParts parts, int64_t nchunk_b, float *__restrict__ grads) {
    constexpr int64_t kOffB[4] = {off_b(0), off_b(1), off_b(2), off_b(3)};
    __shared__ double red[kRedBLanes][kRedBEntries];
    const int le = threadIdx.x % kRedBEntries, cl = threadIdx.x / kRedBEntries;
    const int e = (int)blockIdx.x * kRedBEntries + le;
    const int l = e < 3 * kHid ? e / kHid : 3, m = e - l * kHid, MP = mpad(l);
    double s0 = 0.0, s1 = 0.0;
    if (e < kRedBias) {
        const double *p = parts.b[l] + m;
        int64_t c = cl;
        for (; c + kRedBLanes < nchunk_b; c += 2 * kRedBLanes) {
            s0 += p[c * MP];
            s1 += p[(c + kRedBLanes) * MP];
        }
        if (c < nchunk_b) s0 += p[c * MP];
    }
    red[cl][le] = s0 + s1;
    __syncthreads();
    if (cl == 0 && e < kRedBias) {
        double t = 0.0;
        for (int q = 0; q < kRedBLanes; ++q) t += red[q][le];
        grads[kOffB[l] + m] = (float)t;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_loss(const double *__restrict__ part, int64_t n, float *__restrict__ out) {
    __shared__ double red[kWavesPerBlock];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) v += part[i];
    v = block_sum(v, red);
    if (threadIdx.x == 0) out[0] = (float)v;
}

__global__ __launch_bounds__(kBlock) void k_output(const float *__restrict__ y16, int64_t B, float *__restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < B * 3) y[e] = y16[(e / 3) * 16 + e % 3];
}

// Column statistics: pass 0 sums x, pass 1 sums (x - mean)^2, per chunk of rows.
__global__ __launch_bounds__(kBlock) void k_colsum(const float *__restrict__ x, int64_t n, int cols, int64_t rows_per,
                                                   const double *__restrict__ mean, double *__restrict__ part) {
    const int c = threadIdx.x;
    if (c >= cols) return;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = (r0 + rows_per < n) ? r0 + rows_per : n;
    const double mu = mean ? mean[c] : 0.0;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double v = (double)x[r * cols + c] - mu;
        s += mean ? v * v : v;
    }
    part[(int64_t)blockIdx.x * cols + c] = s;
}

__global__ __launch_bounds__(kBlock) void k_colfinish(const double *__restrict__ part, int64_t nchunk, int cols,
                                                      int64_t n, int sq, double *__restrict__ out) {
    const int c = threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    for (int64_t k = 0; k < nchunk; ++k) s += part[k * cols + c];
    out[c] = sq ? sqrt(s / (double)n) : s / (double)n;
}

// ---------------------------------------------------------------------------
// Features of given particles from the bulk fields (training pairs)
// ---------------------------------------------------------------------------
// feat[j] = the 193 raw features of particle i = sel[j] (or j): per stencil cell
// (dz, dy, dx in -1..1, dx fastest, clamped at the walls) eps = 1 - phi, U, G,
// neighbours minus the centre cell; offsets x * n / L - i; d * n_x / L_x.
// u_bulk[j] = bulk trilinear velocity; resid[j] = u_fine[i] - u_bulk[j].
__global__ __launch_bounds__(kBlock) void k_features(Geo<float> g, int64_t n, const float *__restrict__ pos,
                                                     const float *__restrict__ diam, const float *__restrict__ phi,
                                                     const float *__restrict__ U, const float *__restrict__ G,
                                                     const float *__restrict__ u_fine, const int32_t *__restrict__ sel,
                                                     int64_t nsel, float *__restrict__ feat,
                                                     float *__restrict__ u_bulk, float *__restrict__ resid) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nsel) return;
    int64_t i = sel ? (int64_t)sel[j] : j;
    if (i < 0 || i >= n) i = 0;   // documented: entries must be in range; keeps loads in bounds
    int o = 0;
    const float x = clamp_coord(pos[3 * i + 0], g.L[0], o), y = clamp_coord(pos[3 * i + 1], g.L[1], o),
                z = clamp_coord(pos[3 * i + 2], g.L[2], o);
    const int ix = cell_axis(x, g.sb[0], g.nb[0]), iy = cell_axis(y, g.sb[1], g.nb[1]),
              iz = cell_axis(z, g.sb[2], g.nb[2]);
    const int64_t nx = g.nb[0], nxy = (int64_t)g.nb[0] * g.nb[1], nc = g.ncell;
    const int64_t c0 = ix + nx * iy + nxy * iz;
    float cen[7] = {1.f - phi[c0], U[c0], U[nc + c0], U[2 * nc + c0], G[c0], G[nc + c0], G[2 * nc + c0]};
    float *out = feat + j * kFeat;
    int col = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int cx = clampi(ix + dx, g.nb[0]), cy = clampi(iy + dy, g.nb[1]), cz = clampi(iz + dz, g.nb[2]);
                const int64_t c = cx + nx * cy + nxy * cz;
                const float v[7] = {1.f - phi[c], U[c], U[nc + c], U[2 * nc + c], G[c], G[nc + c], G[2 * nc + c]};
                const bool centre = (dx == 0 && dy == 0 && dz == 0);
                for (int k = 0; k < 7; ++k) out[col++] = centre ? cen[k] : v[k] - cen[k];
            }
    out[col++] = x * g.sb[0] - (float)ix;
    out[col++] = y * g.sb[1] - (float)iy;
    out[col++] = z * g.sb[2] - (float)iz;
    out[col++] = diam[i] * g.sb[0];
    if (u_bulk || resid) {
        const Axis<float> bx = cic_axis(x, g.sb[0], g.nb[0]);
        const Axis<float> by = cic_axis(y, g.sb[1], g.nb[1]);
        const Axis<float> bz = cic_axis(z, g.sb[2], g.nb[2]);
        const int inx = g.nb[0];
        float ub[3];
        for (int a = 0; a < 3; ++a) ub[a] = trilin_pairs(U + a * nc, bx, by, bz, inx, nxy);
        if (u_bulk)
            for (int a = 0; a < 3; ++a) u_bulk[3 * j + a] = ub[a];
        if (resid && u_fine)
            for (int a = 0; a < 3; ++a) resid[3 * j + a] = u_fine[3 * i + a] - ub[a];
    }
}

// ---------------------------------------------------------------------------
// In-step inference: packed bulk features, fused gather + four-layer chain,
// sampled check with fine fallback
// ---------------------------------------------------------------------------
// fgrid[2c] = (1 - phi, U_x, U_y, U_z), fgrid[2c+1] = (G_x, G_y, G_z, 0); G is
// also written to the bulk gradient output (same values as the source stage).
__global__ __launch_bounds__(kBlock) void k_pack(StepArgs<float> a) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= a.g.ncell) return;
    int cx, cy, cz;
    decode_cell(c, a.g.nb, cx, cy, cz);
    float gr[3];
    gradient_at(c, cx, cy, cz, a.g.nb, a.g.hb, a.P, a.Plo, gr);
    const int64_t nc = a.g.ncell;
    for (int k = 0; k < 3; ++k) a.G[k * nc + c] = gr[k];
    a.fgrid[2 * c] = make_float4(1.f - a.phi[c], a.U[c], a.U[nc + c], a.U[2 * nc + c]);
    a.fgrid[2 * c + 1] = make_float4(gr[0], gr[1], gr[2], 0.f);
}

constexpr int kInfWaves = 8;                    // waves per workgroup (two per SIMD: the LDS and 256 VGPRs per wave)
constexpr int kInfTiles = 2;                    // 16-particle tiles per wave and round
constexpr int kInfRows = 16 * kInfTiles;        // particles per wave and round
constexpr int kFrag1 = 8 * 7, kFragH = 8 * 4;   // operand fragments per layer
constexpr int kFrags = kFrag1 + 2 * kFragH + 4;

struct InferLds {
    uint4 frag[kFrags][kWave];    // weight fragments in slot order, 16 B per lane
    float bias[3 * kHid + 16];    // b1, b2, b3, b4 (padded)
    float mean[kK1], inv[kK1];    // standardisation per feature (0 in the padding)
};

// Layer-1 slot (kb, g, i) -> feature index: unit u = 4 kb + g is stencil cell u
// (its 7 channels in slots 0-6) or, for u = 27, the offsets and diameter.
__device__ __forceinline__ int slot_feature(int kb, int g, int i) {
    const int u = 4 * kb + g;
    if (u < 27) return i < 7 ? 7 * u + i : -1;
    return i < 4 ? 189 + i : -1;
}
// Hidden-layer slot (kb, g, i) -> input neuron (result-layout pairing).
__device__ __forceinline__ int slot_hidden(int kb, int g, int i) {
    return 32 * kb + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}

// One layer of the chain for NT tiles: in[t][kb] (KB slot groups) -> 8 row
// blocks (accumulators start at the bias) -> gelu -> out[t][4] in the paired
// slot order.  The slot-group loop is outermost so that the 8 NT accumulators
// form independent MFMA chains (a dependent MFMA waits for its predecessor);
// each weight fragment read from LDS feeds NT products.
template <int NT, int KB>
__device__ __forceinline__ void chain_layer(const InferLds &L, int frag0, const float *bias,
                                            const uint4 (&in)[NT][KB], uint4 (&out)[NT][4], int lane, int g) {
    f32x4 acc[8][NT];
#pragma unroll
    for (int mb = 0; mb < 8; ++mb) {
        const int m0 = 16 * mb + 4 * g;
        const f32x4 b = {bias[m0], bias[m0 + 1], bias[m0 + 2], bias[m0 + 3]};
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[mb][t] = b;
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int mb = 0; mb < 8; ++mb) {
            const bf16x8 w = as_bf16x8(L.frag[frag0 + mb * KB + kb][lane]);
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[mb][t] = mma(w, as_bf16x8(in[t][kb]), acc[mb][t]);
        }
#pragma unroll
    for (int mb = 0; mb < 8; ++mb)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const uint32_t lo = pack2(gelu(acc[mb][t][0]), gelu(acc[mb][t][1]));
            const uint32_t hi = pack2(gelu(acc[mb][t][2]), gelu(acc[mb][t][3]));
            if (mb & 1) {
                out[t][mb >> 1].z = lo;
                out[t][mb >> 1].w = hi;
            } else {
                out[t][mb >> 1].x = lo;
                out[t][mb >> 1].y = hi;
            }
        }
}

// Bulk trilinear velocity and void fraction at a particle from the packed
// features (fgrid[2c] = (eps_c, U_c)): u_bulk = sum_c w_pc U_c and
// eps_p = sum_c w_pc eps_c with the deposition weights (CIC or NGP).  Where the
// particle solid fraction exceeds phi_fp64 the sum is taken in FP64 (eps_c =
// 1 - phi_c is exact for phi_c >= 1/2, where it matters).
__device__ __forceinline__ float4 bulk_sample_packed(const StepArgs<float> &a, const float4 &q) {
    const Geo<float> &g = a.g;
    const Axis<float> bx = cic_axis(q.x, g.sb[0], g.nb[0]);
    const Axis<float> by = cic_axis(q.y, g.sb[1], g.nb[1]);
    const Axis<float> bz = cic_axis(q.z, g.sb[2], g.nb[2]);
    const int64_t nx = g.nb[0], nxy = (int64_t)g.nb[0] * g.nb[1];
    const int64_t zl = bz.lo * nxy, zh = bz.hi * nxy, yl = by.lo * nx, yh = by.hi * nx;
    const float4 c000 = a.fgrid[2 * (zl + yl + bx.lo)], c001 = a.fgrid[2 * (zl + yl + bx.hi)];
    const float4 c010 = a.fgrid[2 * (zl + yh + bx.lo)], c011 = a.fgrid[2 * (zl + yh + bx.hi)];
    const float4 c100 = a.fgrid[2 * (zh + yl + bx.lo)], c101 = a.fgrid[2 * (zh + yl + bx.hi)];
    const float4 c110 = a.fgrid[2 * (zh + yh + bx.lo)], c111 = a.fgrid[2 * (zh + yh + bx.hi)];
    const float sx = 1.f - bx.t, sy = 1.f - by.t, sz = 1.f - bz.t;
    auto tri = [&](float v000, float v001, float v010, float v011, float v100, float v101, float v110, float v111) {
        return sz * (sy * (sx * v000 + bx.t * v001) + by.t * (sx * v010 + bx.t * v011)) +
               bz.t * (sy * (sx * v100 + bx.t * v101) + by.t * (sx * v110 + bx.t * v111));
    };
    float4 r;
    r.x = tri(c000.y, c001.y, c010.y, c011.y, c100.y, c101.y, c110.y, c111.y);
    r.y = tri(c000.z, c001.z, c010.z, c011.z, c100.z, c101.z, c110.z, c111.z);
    r.z = tri(c000.w, c001.w, c010.w, c011.w, c100.w, c101.w, c110.w, c111.w);
    if (a.cic) {
        const float e = tri(c000.x, c001.x, c010.x, c011.x, c100.x, c101.x, c110.x, c111.x);
        if (1.f - e > a.phi_fp64) {
            const double gx = (double)q.x * (double)g.sb[0] - 0.5, gy = (double)q.y * (double)g.sb[1] - 0.5,
                         gz = (double)q.z * (double)g.sb[2] - 0.5;
            const double tx = gx - floor(gx), ty = gy - floor(gy), tz = gz - floor(gz);
            const double ux = 1.0 - tx, uy = 1.0 - ty, uz = 1.0 - tz;
            r.w = (float)(uz * (uy * (ux * (double)c000.x + tx * (double)c001.x) +
                                ty * (ux * (double)c010.x + tx * (double)c011.x)) +
                          tz * (uy * (ux * (double)c100.x + tx * (double)c101.x) +
                                ty * (ux * (double)c110.x + tx * (double)c111.x)));
        } else {
            r.w = e;
        }
    } else {
        const int ix = cell_axis(q.x, g.sb[0], g.nb[0]), iy = cell_axis(q.y, g.sb[1], g.nb[1]),
                  iz = cell_axis(q.z, g.sb[2], g.nb[2]);
        r.w = a.fgrid[2 * (ix + nx * iy + nxy * iz)].x;
    }
    return r;
}

// Standardised layer-1 inputs of one particle (clamped position and diameter q,
// containing cell c0; zero when not valid) for lane group g: x[kb] holds unit
// 4 kb + g.
__device__ __forceinline__ void gather_features(const StepArgs<float> &a, const InferLds &L, const float4 &q,
                                                int64_t c0, bool valid, int g, uint4 (&x)[7]) {
    const Geo<float> &geo = a.g;
    const int64_t nx = geo.nb[0], nxy = (int64_t)geo.nb[0] * geo.nb[1];
    if (c0 < 0 || c0 >= geo.ncell) c0 = 0;
    int ix, iy, iz;
    decode_cell(c0, geo.nb, ix, iy, iz);
    // all stencil loads first (one cell per slot group), then the arithmetic
    float4 B0[7], B1[7];
#pragma unroll
    for (int kb = 0; kb < 7; ++kb) {
        const int u = 4 * kb + g;
        const int uu = u < 27 ? u : 13;
        const int dx = uu % 3 - 1, dy = (uu / 3) % 3 - 1, dz = uu / 9 - 1;
        const int64_t c = clampi(ix + dx, geo.nb[0]) + nx * clampi(iy + dy, geo.nb[1]) + nxy * clampi(iz + dz, geo.nb[2]);
        B0[kb] = a.fgrid[2 * c];
        B1[kb] = a.fgrid[2 * c + 1];
    }
    const float4 A0 = a.fgrid[2 * c0], A1 = a.fgrid[2 * c0 + 1];
#pragma unroll
    for (int kb = 0; kb < 7; ++kb) {
        const int u = 4 * kb + g;
        float v[8];
        int f0, nv;
        if (u < 27) {
            const bool centre = (u == 13);
            v[0] = centre ? A0.x : B0[kb].x - A0.x;
            v[1] = centre ? A0.y : B0[kb].y - A0.y;
            v[2] = centre ? A0.z : B0[kb].z - A0.z;
            v[3] = centre ? A0.w : B0[kb].w - A0.w;
            v[4] = centre ? A1.x : B1[kb].x - A1.x;
            v[5] = centre ? A1.y : B1[kb].y - A1.y;
            v[6] = centre ? A1.z : B1[kb].z - A1.z;
            v[7] = 0.f;
            f0 = 7 * u;
            nv = 7;
        } else {
            v[0] = q.x * geo.sb[0] - (float)ix;
            v[1] = q.y * geo.sb[1] - (float)iy;
            v[2] = q.z * geo.sb[2] - (float)iz;
            v[3] = q.w * geo.sb[0];
            v[4] = v[5] = v[6] = v[7] = 0.f;
            f0 = 189;
            nv = 4;
        }
        float xs[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) xs[i] = (i < nv && valid) ? (v[i] - L.mean[f0 + i]) * L.inv[f0 + i] : 0.f;
        x[kb] = make_uint4(pack2(xs[0], xs[1]), pack2(xs[2], xs[3]), pack2(xs[4], xs[5]), pack2(xs[6], xs[7]));
    }
}

// Persistent: each workgroup takes one contiguous range of the sorted particles
// (neighbouring cells: the stencil loads hit L1/L2), each wave kInfRows particles
// per round.  Lane (n, g) gathers, for tile t and slot group kb, unit 4 kb + g of
// particle 16 t + n; lanes with g < kInfTiles then finish particle 16 g + n:
// u = u_bulk + s * y and eps_p (both from the packed features), written to
// uf4[id].
__global__ __launch_bounds__(kInfWaves * kWave) void k_infer(StepArgs<float> a) {
    __shared__ InferLds L;
    constexpr int NT = kInfTiles;
    const int lane = lane_id(), n = lane & 15, g = lane >> 4, wave = threadIdx.x >> 6;
    const MlpNet &net = a.net;
    // weights into LDS in slot order
    for (int e = threadIdx.x; e < kFrags * kWave * 8; e += kInfWaves * kWave) {
        const int f = e >> 9, ln = (e >> 3) & 63, i = e & 7;
        const int r = ln & 15, gg = ln >> 4;
        uint16_t v = 0;
        if (f < kFrag1) {
            const int mb = f / 7, kb = f % 7;
            const int k = slot_feature(kb, gg, i);
            if (k >= 0) v = net.wt[0][(16 * mb + r) * kpad(0) + k];
        } else if (f < kFrag1 + 2 * kFragH) {
            const int l = (f < kFrag1 + kFragH) ? 1 : 2;
            const int ff = f - kFrag1 - (l - 1) * kFragH;
            const int mb = ff / 4, kb = ff % 4;
            v = net.wt[l][(16 * mb + r) * kpad(l) + slot_hidden(kb, gg, i)];
        } else {
            const int kb = f - kFrag1 - 2 * kFragH;
            v = net.wt[3][r * kpad(3) + slot_hidden(kb, gg, i)];
        }
        reinterpret_cast<uint16_t *>(&L.frag[f][ln])[i] = v;
    }
    for (int e = threadIdx.x; e < 3 * kHid + 16; e += kInfWaves * kWave) {
        const int l = e / kHid, m = e % kHid;
        constexpr int64_t kB0 = off_b(0), kB1 = off_b(1), kB2 = off_b(2), kB3 = off_b(3);
        const int64_t ob = l == 0 ? kB0 : (l == 1 ? kB1 : kB2);
        L.bias[e] = (l < 3) ? net.params[ob + m] : (m < kOut ? net.params[kB3 + m] : 0.f);
    }
    for (int e = threadIdx.x; e < kK1; e += kInfWaves * kWave) {
        L.mean[e] = net.mean_inv[e];
        L.inv[e] = net.mean_inv[kK1 + e];
    }
    __syncthreads();

    const int64_t per = ((a.n + gridDim.x - 1) / gridDim.x + kInfRows - 1) / kInfRows * kInfRows;
    const int64_t s_begin = (int64_t)blockIdx.x * per;
    const int64_t s_end = (s_begin + per < a.n) ? s_begin + per : a.n;
    for (int64_t base = s_begin + (int64_t)wave * kInfRows; base < s_end; base += kInfWaves * kInfRows) {
        float4 q[NT];
        int64_t c[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            int64_t s = base + 16 * t + n;
            s = s < s_end ? s : base;
            q[t] = a.sp[s];
            c[t] = a.keys[s];
        }
        // the particle this lane finishes (tile g): its bulk velocity, void
        // fraction and id are fetched first so that their loads overlap the chain
        const int64_t so = base + 16 * g + n;
        const bool own = (g < NT) && so < s_end;
        float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
        int64_t p = 0;
        if (own) {
            float4 qo = q[0];
#pragma unroll
            for (int t = 1; t < NT; ++t)
                if (g == t) qo = q[t];
            r = bulk_sample_packed(a, qo);
            p = a.perm[so];
            if (p < 0 || p >= a.n) p = 0;
        }
        uint4 x[NT][7];
#pragma unroll
        for (int t = 0; t < NT; ++t) gather_features(a, L, q[t], c[t], base + 16 * t + n < s_end, g, x[t]);
        uint4 h1[NT][4], h2[NT][4];
        chain_layer<NT, 7>(L, 0, L.bias, x, h1, lane, g);
        chain_layer<NT, 4>(L, kFrag1, L.bias + kHid, h1, h2, lane, g);
        chain_layer<NT, 4>(L, kFrag1 + kFragH, L.bias + 2 * kHid, h2, h1, lane, g);
        f32x4 y[NT];
        const f32x4 b4 = {L.bias[3 * kHid], L.bias[3 * kHid + 1], L.bias[3 * kHid + 2], 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) y[t] = b4;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 w = as_bf16x8(L.frag[kFrag1 + 2 * kFragH + kb][lane]);
#pragma unroll
            for (int t = 0; t < NT; ++t) y[t] = mma(w, as_bf16x8(h1[t][kb]), y[t]);
        }
        // lane (n, 0) holds the 3 outputs of particle 16 t + n in y[t]
        float yo[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float v = __shfl(y[t][j], n, kWave);
                if (t == g) yo[j] = v;
            }
        if (own) {
            r.x += net.scale[0] * yo[0];
            r.y += net.scale[1] * yo[1];
            r.z += net.scale[2] * yo[2];
            a.uf4[p] = r;
        }
    }
}

// Bricks of 8x8x8 bulk cells, one wave each.  The checked sample is every
// particle with id mod period = step mod period; where its relative L2 error
// against the fine lookup exceeds tol, every particle of the brick takes the
// fine lookup.  The brick's 64 (z, y) rows are one lane each: their sorted
// ranges are loaded at once and prefix-summed across the wave, and the brick's
// particles are then processed 64 at a time in that flattened order.  Per
// workgroup: fallback count, sampled squared error and reference, sample count
// (FP64 partials, fixed order).
constexpr int kBrick = 8;

__global__ __launch_bounds__(kBlock) void k_check(StepArgs<float> a) {
    static_assert(kBrick * kBrick == kWave, "one lane per (z, y) row of a brick");
    __shared__ double red[kWavesPerBlock];
    __shared__ int32_t pre[kWavesPerBlock][kWave + 1];   // particles before each row (exclusive prefix)
    __shared__ int64_t row0[kWavesPerBlock][kWave];      // first sorted position of each row
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int64_t brick = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    const Geo<float> &geo = a.g;
    double err = 0.0, ref = 0.0, ns = 0.0, nfall = 0.0;
    if (brick < a.n_bricks && a.n > 0) {   // uniform over the wave
        const int bx = (geo.nb[0] + kBrick - 1) / kBrick, by = (geo.nb[1] + kBrick - 1) / kBrick;
        const int ox = (int)(brick % bx) * kBrick, oy = (int)((brick / bx) % by) * kBrick,
                  oz = (int)(brick / ((int64_t)bx * by)) * kBrick;
        const int wx = (ox + kBrick < geo.nb[0]) ? kBrick : geo.nb[0] - ox;
        // lane r owns row (dz, dy) = (r / 8, r % 8): its particles are the
        // contiguous sorted range of cells ox .. ox + wx - 1 of that row
        const int dz = lane / kBrick, dy = lane % kBrick;
        int64_t s0 = 0, s1 = 0;
        if (oz + dz < geo.nb[2] && oy + dy < geo.nb[1]) {
            const int64_t c0 = ox + (int64_t)geo.nb[0] * ((oy + dy) + (int64_t)geo.nb[1] * (oz + dz));
            s0 = seg_clamp(a.start[c0], a.n);
            s1 = seg_clamp(a.start[c0 + wx], a.n);
        }
        int32_t incl = (int32_t)(s1 - s0);   // inclusive prefix over the lanes (rows in order)
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int32_t v = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += v;
        }
        pre[wave][lane + 1] = incl;
        if (lane == 0) pre[wave][0] = 0;
        row0[wave][lane] = s0;
        wave_sync();
        const int32_t total = pre[wave][kWave];
        // flattened index j -> row (last r with pre[r] <= j) -> sorted position
        auto position = [&](int32_t j) {
            int lo = 0, hi = kWave;   // pre[lo] <= j < pre[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pre[wave][mid] <= j) lo = mid;
                else hi = mid;
            }
            return row0[wave][lo] + (j - pre[wave][lo]);
        };
        const int64_t period = a.mlp_period, phase = ((a.step % period) + period) % period;
        // kU particles of a lane per round: their ids are loaded together (one
        // round trip instead of kU), then taken in the lane's order j
        constexpr int kU = 4;
        for (int32_t j0 = lane; j0 < total; j0 += kU * kWave) {
            int64_t s[kU], p[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int32_t j = j0 + u * kWave;
                s[u] = position(j < total ? j : j0);
                p[u] = a.perm[s[u]];
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (j0 + u * kWave >= total) break;
                int64_t pu = p[u];
                if (pu < 0 || pu >= a.n) pu = 0;
                if (pu % period != phase) continue;
                float ux, uy, uz;
                fine_velocity(a.sp[s[u]], a, ux, uy, uz);
                const float4 m = a.uf4[pu];
                const double ex = (double)m.x - ux, ey = (double)m.y - uy, ez = (double)m.z - uz;
                err += ex * ex + ey * ey + ez * ez;
                ref += (double)ux * ux + (double)uy * uy + (double)uz * uz;
                ns += 1.0;
            }
        }
        const double terr = wave_sum(err), tref = wave_sum(ref), tns = wave_sum(ns);
        const double tol = (double)a.mlp_tol;
        if (tns > 0.0 && terr > tol * tol * tref) {
            for (int32_t j = lane; j < total; j += kWave) {
                const int64_t s = position(j);
                int64_t p = a.perm[s];
                if (p < 0 || p >= a.n) p = 0;
                float4 m = a.uf4[p];
                fine_velocity(a.sp[s], a, m.x, m.y, m.z);
                a.uf4[p] = m;
                nfall += 1.0;
            }
        }
    }
    const double vals[4] = {nfall, err, ref, ns};
    const int slots[4] = {SL_NFALL, SL_MLPERR, SL_MLPREF, SL_MLPSAMP};
    for (int k = 0; k < 4; ++k) {
        const double t = block_sum(vals[k], red);
        if (threadIdx.x == 0) a.part[slots[k] * a.part_stride + blockIdx.x] = t;
    }
}

}  // namespace mlp

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
int64_t bricks_of(const int nb[3]) {
    int64_t b = 1;
    for (int a = 0; a < 3; ++a) b *= (nb[a] + mlp::kBrick - 1) / mlp::kBrick;
    return b;
}
int64_t mlp_check_blocks(int64_t n_bricks) { return (n_bricks + kWavesPerBlock - 1) / kWavesPerBlock; }

void launch_mlp_pack(const StepArgs<float> &a, hipStream_t st) {
    hipLaunchKernelGGL(mlp::k_pack, dim3((unsigned)((a.g.ncell + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a);
}

void launch_mlp_infer(const StepArgs<float> &a, hipStream_t st) {
    if (a.n <= 0) return;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu < 1) ncu = 1;
    // one workgroup per compute unit, or fewer for small inputs
    const int64_t rounds = (a.n + mlp::kInfRows - 1) / mlp::kInfRows;
    int64_t grid = ncu;
    if (grid * mlp::kInfWaves > rounds) grid = (rounds + mlp::kInfWaves - 1) / mlp::kInfWaves;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(mlp::k_infer, dim3((unsigned)grid), dim3(mlp::kInfWaves * kWave), 0, st, a);
}

void launch_mlp_check(const StepArgs<float> &a, hipStream_t st) {
    hipLaunchKernelGGL(mlp::k_check, dim3((unsigned)mlp_check_blocks(a.n_bricks)), dim3(kBlock), 0, st, a);
}

namespace mlp {

static WPtrs wptrs(const NetBufs &net) {
    WPtrs w;
    for (int l = 0; l < 4; ++l) {
        w.wt[l] = net.wt[l];
        w.wn[l] = net.wn[l];
        w.wtp[l] = net.wtp[l];
        w.wnp[l] = net.wnp[l];
    }
    return w;
}

static unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_cast(const NetBufs &net, hipStream_t st) {
    hipLaunchKernelGGL(k_cast, dim3(blocks(kNParam)), dim3(kBlock), 0, st, net.params, wptrs(net));
    return hipGetLastError();
}

hipError_t launch_adam(const NetBufs &net, const float *grads, float lr, float b1, float omb1, float b2, float omb2,
                       float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(blocks(kNParam)), dim3(kBlock), 0, st, grads, net.params, net.m, net.v, wptrs(net),
                       lr, b1, omb1, b2, omb2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_standardise(const float *feat, int64_t B, const float *mean_inv, uint16_t *x0, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_standardise, dim3((unsigned)((B + kStdRows - 1) / kStdRows)), dim3(kBlock), 0, st, feat, B,
                       mean_inv, x0);
    return hipGetLastError();
}

static unsigned tile_blocks(int64_t B) { return (unsigned)(((B + 15) / 16 + kWavesPerBlock - 1) / kWavesPerBlock); }

hipError_t launch_forward(const NetBufs &net, const TrainBufs &tb, int64_t B, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    const dim3 gr(tile_blocks(B)), bl(kBlock);
    const float *p = net.params;
    hipLaunchKernelGGL((k_dense<7, 8, false>), gr, bl, 0, st, tb.x0, net.wt[0], p + off_b(0), kHid, B, nullptr, tb.h[0]);
    hipLaunchKernelGGL((k_dense<4, 8, false>), gr, bl, 0, st, tb.h[0], net.wt[1], p + off_b(1), kHid, B, nullptr, tb.h[1]);
    hipLaunchKernelGGL((k_dense<4, 8, false>), gr, bl, 0, st, tb.h[1], net.wt[2], p + off_b(2), kHid, B, nullptr, tb.h[2]);
    hipLaunchKernelGGL((k_dense<4, 1, true>), gr, bl, 0, st, tb.h[2], net.wt[3], p + off_b(3), kOut, B, tb.y, nullptr);
    return hipGetLastError();
}

hipError_t launch_gradients(const NetBufs &net, const TrainBufs &tb, const float *feat, const float *resid,
                            const int32_t *idx, int64_t nrows, int64_t B, const float inv_scale[3], float *grads,
                            float *loss, hipStream_t st) {
    const dim3 bl(kBlock);
    TrainArgs a;
    a.feat = feat;
    a.resid = resid;
    a.idx = idx;
    a.nrows = nrows;
    a.B = B;
    a.mean_inv = net.mean_inv;
    for (int j = 0; j < 3; ++j) a.is[j] = inv_scale[j];
    a.inv_b = (float)(1.0 / (double)B);
    a.params = net.params;
    a.wt0 = net.wt[0];
    for (int l = 0; l < 4; ++l) {
        a.wtp[l] = net.wtp[l];
        a.wnp[l] = net.wnp[l];
        a.part_b[l] = tb.part_b[l];
    }
    a.tr = tb.tr;
    a.loss_part = tb.loss_part;
    if (B <= 0 || B % kTrainGroupRows != 0) return hipErrorInvalidValue;   // every workgroup has both tiles
    const unsigned nt = (unsigned)n_train_groups(B);
    hipLaunchKernelGGL(k_train_tile, dim3(nt), dim3(kTrainThreads), 0, st, a);
    const unsigned nc = (unsigned)n_chunks(B);
    const dim3 bw(kWgradWaves * kWave);
    WgradParts wp;
    for (int l = 0; l < 4; ++l) wp.w[l] = tb.part_w[l];
    hipLaunchKernelGGL(k_wgrad, dim3(nc, 4), bw, 0, st, tb.tr, B, wp);
    GradParts parts;
    for (int l = 0; l < 4; ++l) {
        parts.w[l] = tb.part_w[l];
        parts.b[l] = tb.part_b[l];
    }
    hipLaunchKernelGGL(k_reduce_w, dim3((unsigned)((kRedTotal + kRedEntries - 1) / kRedEntries)), bl, 0, st, parts,
                       (int64_t)nc, grads);
    hipLaunchKernelGGL(k_reduce_b, dim3((unsigned)((kRedBias + kRedBEntries - 1) / kRedBEntries)), dim3(kRedBThreads), 0,
                       st, parts, (int64_t)nt, grads);
    if (loss) hipLaunchKernelGGL(k_sum_loss, dim3(1), bl, 0, st, tb.loss_part, B / 16, loss);
    return hipGetLastError();
}

hipError_t launch_output(const TrainBufs &tb, int64_t B, float *y, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_output, dim3(blocks(B * 3)), dim3(kBlock), 0, st, tb.y, B, y);
    return hipGetLastError();
}

hipError_t launch_column_stats(const float *x, int64_t n, int cols, double *part, int64_t nchunk, double *mean,
                               double *std, hipStream_t st) {
    const int64_t rows_per = (n + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)nchunk), dim3(kBlock), 0, st, x, n, cols, rows_per, nullptr, part);
    hipLaunchKernelGGL(k_colfinish, dim3(1), dim3(kBlock), 0, st, part, nchunk, cols, n, 0, mean);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)nchunk), dim3(kBlock), 0, st, x, n, cols, rows_per, mean, part);
    hipLaunchKernelGGL(k_colfinish, dim3(1), dim3(kBlock), 0, st, part, nchunk, cols, n, 1, std);
    return hipGetLastError();
}

hipError_t launch_features(const int nb[3], const double box[3], int64_t n, const float *pos, const float *diam,
                           const float *phi, const float *U, const float *G, const float *u_fine,
                           const int32_t *sel, int64_t nsel, float *feat, float *u_bulk, float *resid,
                           hipStream_t st) {
    if (nsel <= 0) return hipSuccess;
    Geo<float> g;
    for (int a = 0; a < 3; ++a) {
        g.nb[a] = nb[a];
        g.nf[a] = nb[a];
        g.L[a] = (float)box[a];
        g.sb[a] = (float)((double)nb[a] / box[a]);
        g.sf[a] = g.sb[a];
        g.hb[a] = (float)(box[a] / (double)nb[a]);
    }
    g.ncell = (int64_t)nb[0] * nb[1] * nb[2];
    g.nfine = g.ncell;
    g.vb = (box[0] / nb[0]) * (box[1] / nb[1]) * (box[2] / nb[2]);
    g.vf = g.vb;
    g.inv_vb = (float)(1.0 / g.vb);
    hipLaunchKernelGGL(k_features, dim3(blocks(nsel)), dim3(kBlock), 0, st, g, n, pos, diam, phi, U, G, u_fine, sel, nsel,
                       feat, u_bulk, resid);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace cpl
