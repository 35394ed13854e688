// Fourier-feature MLP surrogate of the scattered field A(theta, phi, f):
// training and inference kernels for gfx950.
//
// The dense layers are bf16 x bf16 -> fp32 matrix products on the matrix
// cores (v_mfma_f32_32x32x16_bf16) with the bias, the activation and the
// bf16 rounding fused into the epilogue.  One kernel computes
// C[m][n] = sum_k A[m][k] B[n][k] with both operands stored k-contiguous,
// which serves the forward product (A = activations, B = weights), the
// backward product for the input gradient (B = transposed weights) and the
// weight gradient (A = transposed output gradient, B = transposed
// activations; the forward and backward epilogues write those transposes).
// A 256-thread block owns a 64 x 128 tile of C; each wave owns a 32 x 64
// sub-tile (two 32 x 32 MFMA blocks) and walks k in steps of 16.
//
// Fragment layout of v_mfma_f32_32x32x16_bf16: lane l supplies row l % 32
// of A (and of B), elements k0 + 8 (l / 32) .. + 7 (the same k split for
// both operands, so the product does not depend on how the hardware orders
// k); accumulator register r of lane l holds C[8 (r / 4) + 4 (l / 32) +
// r % 4][l % 32].
//
// Rounding points (fp32 -> bf16, nearest-even, written out below): the
// Fourier features, every hidden activation, and the activation-gradient
// operand of the two backward products.  Reductions over the batch (weight
// and bias gradients, the loss) run in a fixed order: results are bitwise
// reproducible.
#include <cmath>
#include <type_traits>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// float32 -> bf16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t to_bf16x2(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{lo, hi}), bf16x2));
}

__device__ __forceinline__ uint16_t to_bf16(float x) { return static_cast<uint16_t>(to_bf16x2(x, 0.0f)); }

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// SiLU through the logistic function sigma(z) = 1 / (1 + 2^(-z log2 e)),
// with the hardware base-2 exponential and reciprocal (about 1 ulp each;
// the activations are rounded to bf16 afterwards).  At z -> -inf the
// exponential overflows to +inf and sigma to 0, so SiLU -> -0.
__device__ __forceinline__ float sigmoid_f(float z)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

template <int kAct>
__device__ __forceinline__ float act_t(float z)
{
    if constexpr (kAct == kActSilu) return z * sigmoid_f(z);
    else return fmaxf(z, 0.0f);
}

__device__ __forceinline__ float act_f(float z, int kind) { return kind == kActSilu ? act_t<kActSilu>(z) : act_t<kActRelu>(z); }

__device__ __forceinline__ float act_d(float z, int kind)
{
    if (kind == kActSilu) {
        const float s = sigmoid_f(z);
        return s * (1.0f + z * (1.0f - s));
    }
    return z > 0.0f ? 1.0f : 0.0f;
}

// Fourier features of one point: xn = the point mapped to [-1, 1]^3, then
// for feature q (sin 2 pi t, cos 2 pi t) with t = B_q . xn in float64,
// reduced to [-1/2, 1/2] revolutions before the hardware float32 sine and
// cosine (which take revolutions, so no rounded 2 pi factor enters; their
// error on [-1/2, 1/2] is about 1.3e-7 absolute, below a float32 ulp of 1).
__device__ __forceinline__ double norm_coord(const double *p, const MlpNorm &nm, int c)
{
    return 2.0 * (p[c] - nm.lo[c]) / (nm.hi[c] - nm.lo[c]) - 1.0;
}

__device__ __forceinline__ void ff_pair(const double *xn, const float *Bq, uint16_t &hs, uint16_t &hc)
{
    double t = 0.0;
    for (int c = 0; c < 3; ++c) t += static_cast<double>(Bq[c]) * xn[c];
    const float fr = static_cast<float>(t - rint(t));
    hs = to_bf16(__builtin_amdgcn_sinf(fr));  // v_sin_f32 / v_cos_f32 take revolutions
    hc = to_bf16(__builtin_amdgcn_cosf(fr));
}

// ---------------------------------------------------------------- GEMM
constexpr int kGemmThreads = 256;
constexpr int kTileM = 64, kTileN = 128, kGemmRing = 4;

// C = A B^T over k (both operands k-contiguous, bf16), 64 x TN tiles (TN =
// 128: one 32 x 64 piece per wave, two accumulators; TN = 64: one 32 x 32
// piece, for products too small to give every CU a 64 x 128 tile); NK > 0:
// exactly NK k steps per block (unrolled), NK = 0: any multiple of 16.  Each
// output element sums k in the same order whatever the tile.
template <int EPI, int NK, int TN = kTileN>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int bx, int by, int bz)
{
    constexpr int NC = TN / 64;  // 32-column accumulators per wave
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m0 = bx * kTileM + (wv & 1) * 32;
    const int n0 = by * TN + (wv >> 1) * (32 * NC);
    const int r = lane & 31, kh = (lane >> 5) * 8;
    // split-K (kEpiF32): block z sums k in [z Kc, (z + 1) Kc) into slice z of fout
    const int kc = g.K / g.ksplit, kb = bz * kc;
    const uint16_t *pa = g.A + static_cast<int64_t>(m0 + r) * g.lda + kh + kb;
    const uint16_t *pb0 = g.B + static_cast<int64_t>(n0 + r) * g.ldb + kh + kb;
    const uint16_t *pb1 = g.B + static_cast<int64_t>(n0 + 32 * (NC - 1) + r) * g.ldb + kh + kb;
    float *fout = g.fout ? g.fout + bz * g.split_stride : nullptr;
    f32x16 acc0 = {}, acc1 = {};
    if constexpr (NK > 0) {
        // NK k steps, unrolled, with the fragments of kGemmRing steps in flight
        bf16x8 ra[kGemmRing], rb0[kGemmRing], rb1[kGemmRing];
#pragma unroll
        for (int u = 0; u < kGemmRing && u < NK; ++u) {
            ra[u] = *reinterpret_cast<const bf16x8 *>(pa + 16 * u);
            rb0[u] = *reinterpret_cast<const bf16x8 *>(pb0 + 16 * u);
            if (NC == 2) rb1[u] = *reinterpret_cast<const bf16x8 *>(pb1 + 16 * u);
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int u = k % kGemmRing;
            const bf16x8 a = ra[u], b0 = rb0[u], b1 = rb1[u];
            if (k + kGemmRing < NK) {
                ra[u] = *reinterpret_cast<const bf16x8 *>(pa + 16 * (k + kGemmRing));
                rb0[u] = *reinterpret_cast<const bf16x8 *>(pb0 + 16 * (k + kGemmRing));
                if (NC == 2) rb1[u] = *reinterpret_cast<const bf16x8 *>(pb1 + 16 * (k + kGemmRing));
            }
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
            if (NC == 2) acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
        }
    } else {
        for (int k0 = 0; k0 < kc; k0 += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(pa + k0);
            const bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(pb0 + k0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
            if (NC == 2) {
                const bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(pb1 + k0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
            }
        }
    }
    // register q holds row m0 + 8 (q / 4) + 4 (lane / 32) + q % 4 of column n:
    // the four rows of a quad are consecutive, so the transposed bf16 copy is
    // written as one 8-byte store per quad
    for (int c = 0; c < NC; ++c) {
        const f32x16 &acc = c ? acc1 : acc0;
        const int n = n0 + 32 * c + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int mq = m0 + 8 * j + 4 * (lane >> 5);
            uint16_t hq[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = mq + i;
                const float v = acc[4 * j + i];
                if (EPI == kEpiHidden) {
                    const float z = v + g.bias[n];
                    if (g.zout) g.zout[static_cast<int64_t>(m) * g.ldz + n] = z;
                    hq[i] = to_bf16(act_f(z, g.act));
                    g.hout[static_cast<int64_t>(m) * g.ldh + n] = hq[i];
                } else if (EPI == kEpiDz) {
                    const float dz = v * act_d(g.zin[static_cast<int64_t>(m) * g.ldzi + n], g.act);
                    g.fout[static_cast<int64_t>(m) * g.ldf + n] = dz;
                    hq[i] = to_bf16(dz);
                    g.hout[static_cast<int64_t>(m) * g.ldh + n] = hq[i];
                } else {
                    fout[static_cast<int64_t>(m) * g.ldf + n] = v;
                }
            }
            if (EPI != kEpiF32 && g.htout) {
                const uint2 w = make_uint2(hq[0] | static_cast<uint32_t>(hq[1]) << 16, hq[2] | static_cast<uint32_t>(hq[3]) << 16);
                *reinterpret_cast<uint2 *>(g.htout + static_cast<int64_t>(n) * g.ldht + mq) = w;
            }
        }
    }
}

template <int EPI, int NK, int TN>
__global__ __launch_bounds__(kGemmThreads) void k_gemm(GemmArgs g)
{
    gemm_tile<EPI, NK, TN>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// ---------------------------------------------------------------- features
// Row m < M: normalised input xn = 2 (x - lo) / (hi - lo) - 1 and features
// sin / cos(2 pi t), t = B xn in float64, reduced to t - rint(t) before the
// float32 sine and cosine.  Rows in [M, Mpad) are zero.
__global__ void k_embed(const double *__restrict__ pts, int64_t M, int64_t Mpad, MlpNorm nm,
                        const float *__restrict__ Bff, int n_ff, uint16_t *__restrict__ h0, uint16_t *__restrict__ h0t)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= Mpad * n_ff) return;
    const int64_t m = i / n_ff;
    const int f = static_cast<int>(i % n_ff);
    uint16_t hs = 0, hc = 0;
    if (m < M) {
        double xn[3];
        for (int c = 0; c < 3; ++c) xn[c] = norm_coord(pts + 3 * m, nm, c);
        ff_pair(xn, Bff + 3 * f, hs, hc);
    }
    const int w = 2 * n_ff;
    h0[m * w + f] = hs;
    h0[m * w + n_ff + f] = hc;
    if (h0t) {
        h0t[static_cast<int64_t>(f) * Mpad + m] = hs;
        h0t[static_cast<int64_t>(n_ff + f) * Mpad + m] = hc;
    }
}

// Training batch: rows m < count are rows idx[m] of the points and of the
// complex targets (the targets divided by the output scale, as 4 reals),
// rows in [count, Mpad) are zero; writes the rows' Fourier features (h0 and
// its transpose) and targets.  *bump (nullable) += 1: the step count of a
// training step (Adam reads it), kept on the device.
__global__ void k_embed_batch(const double *__restrict__ pts, const double *__restrict__ tc,
                              const int32_t *__restrict__ idx, int64_t count, int64_t Mpad, MlpNorm nm,
                              const float *__restrict__ Bff, int n_ff, double inv_scale, uint16_t *__restrict__ h0,
                              uint16_t *__restrict__ h0t, float *__restrict__ tb, int64_t *bump)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (bump && i == 0) *bump += 1;
    if (i >= Mpad * n_ff) return;
    const int64_t m = i / n_ff;
    const int f = static_cast<int>(i % n_ff);
    uint16_t hs = 0, hc = 0;
    int64_t src = 0;
    if (m < count) {
        src = idx[m];
        double xn[3];
        for (int c = 0; c < 3; ++c) xn[c] = norm_coord(pts + 3 * src, nm, c);
        ff_pair(xn, Bff + 3 * f, hs, hc);
    }
    const int w = 2 * n_ff;
    h0[m * w + f] = hs;
    h0[m * w + n_ff + f] = hc;
    h0t[static_cast<int64_t>(f) * Mpad + m] = hs;
    h0t[static_cast<int64_t>(n_ff + f) * Mpad + m] = hc;
    if (f == 0)
        for (int c = 0; c < 4; ++c) tb[4 * m + c] = m < count ? static_cast<float>(tc[4 * src + c] * inv_scale) : 0.f;
}

// ---------------------------------------------------------------- output layer
// 16 rows per 256-thread block, 16 lanes per row (a row of width bf16
// activations read as 16 contiguous pieces).  y = h W_out^T + b_out in
// float32.  Mode 0 (inference): A[m] = scale (y0 + j y1, y2 + j y3) as
// float64.  Mode 1 (training): y, dy = 2 (y - t) / (4 M) (zero for padding
// rows) and a per-block partial of the squared error.
__global__ __launch_bounds__(256) void k_out(const uint16_t *__restrict__ h, int width, const uint16_t *__restrict__ wo,
                                             const float *__restrict__ bo, int64_t M, int64_t Mrows, int mode,
                                             double scale, double *__restrict__ A, const float *__restrict__ tgt,
                                             float *__restrict__ dy, float *__restrict__ partial)
{
    __shared__ float red[16];
    const int row = threadIdx.x >> 4, sub = threadIdx.x & 15;
    const int64_t m = static_cast<int64_t>(blockIdx.x) * 16 + row;
    float y[4] = {0.f, 0.f, 0.f, 0.f};
    if (m < Mrows) {
        const int per = width / 16;
        const bool wide = (per & 7) == 0 && (reinterpret_cast<uintptr_t>(h) & 15) == 0 &&
                          (reinterpret_cast<uintptr_t>(wo) & 15) == 0;
        if (wide) {  // the same sums, 8 activations and 4 x 8 weights per 16-byte load
            for (int k8 = sub * per; k8 < (sub + 1) * per; k8 += 8) {
                const uint4 hv8 = *reinterpret_cast<const uint4 *>(h + m * width + k8);
                uint4 w8[4];
                for (int o = 0; o < 4; ++o) w8[o] = *reinterpret_cast<const uint4 *>(wo + o * width + k8);
                const uint32_t *hw = reinterpret_cast<const uint32_t *>(&hv8);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float hv = from_bf16(static_cast<uint16_t>(hw[j >> 1] >> (16 * (j & 1))));
                    for (int o = 0; o < 4; ++o) {
                        const uint32_t *ww = reinterpret_cast<const uint32_t *>(&w8[o]);
                        y[o] += hv * from_bf16(static_cast<uint16_t>(ww[j >> 1] >> (16 * (j & 1))));
                    }
                }
            }
        } else {
            for (int k = sub * per; k < (sub + 1) * per; ++k) {
                const float hv = from_bf16(h[m * width + k]);
                for (int o = 0; o < 4; ++o) y[o] += hv * from_bf16(wo[o * width + k]);
            }
        }
    }
    for (int off = 8; off >= 1; off >>= 1)
        for (int o = 0; o < 4; ++o) y[o] += __shfl_xor(y[o], off, 16);
    float e2 = 0.f;
    if (sub == 0 && m < Mrows) {
        for (int o = 0; o < 4; ++o) y[o] += bo[o];
        if (mode == 0) {
            if (m < M) {
                A[4 * m + 0] = scale * y[0];
                A[4 * m + 1] = scale * y[1];
                A[4 * m + 2] = scale * y[2];
                A[4 * m + 3] = scale * y[3];
            }
        } else {
            for (int o = 0; o < 4; ++o) {
                const float d = m < M ? y[o] - tgt[4 * m + o] : 0.f;
                e2 += d * d;
                dy[4 * m + o] = m < M ? 2.0f * d / (4.0f * static_cast<float>(M)) : 0.f;
            }
        }
    }
    if (mode == 1) {
        if (sub == 0) red[row] = e2;
        __syncthreads();
        if (threadIdx.x == 0) {
            float s = 0.f;
            for (int q = 0; q < 16; ++q) s += red[q];
            partial[blockIdx.x] = s;
        }
    }
}

// dh = dy W_out (float32, bf16 weights), dz = dh act'(z); writes dz, bf16(dz)
// and its transpose.  One thread per (4 consecutive rows, column), so the
// transposed copy is written 8 bytes at a time (Mrows is a multiple of 64);
// block b of 256.
__device__ __forceinline__ void out_back(const float *__restrict__ dy, const uint16_t *__restrict__ wo, int width,
                                         int64_t Mrows, const float *__restrict__ z, int act, float *__restrict__ dz,
                                         uint16_t *__restrict__ dzb, uint16_t *__restrict__ dzbt, int64_t blk)
{
    const int64_t t = blk * 256 + threadIdx.x;
    if (t >= (Mrows / 4) * width) return;
    const int64_t m0 = 4 * (t / width);
    const int k = static_cast<int>(t % width);
    float wk[4];
    for (int o = 0; o < 4; ++o) wk[o] = from_bf16(wo[o * width + k]);
    uint16_t b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + r, i = m * width + k;
        float dh = 0.f;
        for (int o = 0; o < 4; ++o) dh += dy[4 * m + o] * wk[o];
        const float d = dh * act_d(z[i], act);
        dz[i] = d;
        b[r] = to_bf16(d);
        dzb[i] = b[r];
    }
    *reinterpret_cast<uint2 *>(dzbt + static_cast<int64_t>(k) * Mrows + m0) =
        make_uint2(b[0] | static_cast<uint32_t>(b[1]) << 16, b[2] | static_cast<uint32_t>(b[3]) << 16);
}

// Output-layer gradient partials of rows [64 y, 64 y + 64) (block (x, y)):
// pw[y][o][k] = sum dy[m][o] h[m][k], pb[y][o] = sum dy[m][o]; 256 threads =
// 4 row phases x 64 columns, combined in a fixed order.
__device__ __forceinline__ void out_wgrad_part(const float *__restrict__ dy, const uint16_t *__restrict__ h, int width,
                                               int64_t Mrows, float *__restrict__ pw, float *__restrict__ pb, int bx,
                                               int by)
{
    __shared__ float red[4][5][64];
    const int c = threadIdx.x & 63, t4 = threadIdx.x >> 6;
    const int k = bx * 64 + c;
    const int64_t r0 = static_cast<int64_t>(by) * 64, r1 = min(r0 + 64, Mrows);
    float a[4] = {0.f, 0.f, 0.f, 0.f}, b = 0.f;
    for (int64_t m = r0 + t4; m < r1; m += 4) {
        const float hv = k < width ? from_bf16(h[m * width + k]) : 0.f;
        for (int o = 0; o < 4; ++o) a[o] += dy[4 * m + o] * hv;
        if (c < 4) b += dy[4 * m + c];
    }
    for (int o = 0; o < 4; ++o) red[t4][o][c] = a[o];
    red[t4][4][c] = b;
    __syncthreads();
    if (t4 == 0) {
        if (k < width)
            for (int o = 0; o < 4; ++o)
                pw[(static_cast<int64_t>(by) * 4 + o) * width + k] =
                    ((red[0][o][c] + red[1][o][c]) + red[2][o][c]) + red[3][o][c];
        if (bx == 0 && c < 4)
            pb[static_cast<int64_t>(by) * 4 + c] = ((red[0][4][c] + red[1][4][c]) + red[2][4][c]) + red[3][4][c];
    }
}

// Column-sum partials of rows [64 y, 64 y + 64) of a row-major float32
// matrix (bias gradients), same layout of threads; block (x, y).
__device__ __forceinline__ void colsum_part(const float *__restrict__ x, int64_t rows, int cols,
                                            float *__restrict__ part, int bx, int by)
{
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, t4 = threadIdx.x >> 6;
    const int col = bx * 64 + c;
    const int64_t r0 = static_cast<int64_t>(by) * 64, r1 = min(r0 + 64, rows);
    float sum = 0.f;
    if (col < cols)
        for (int64_t m = r0 + t4; m < r1; m += 4) sum += x[m * cols + col];
    red[t4][c] = sum;
    __syncthreads();
    if (t4 == 0 && col < cols)
        part[static_cast<int64_t>(by) * cols + col] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// out[i] = sum over z of part[z][i].  A block of 256 threads takes 64
// consecutive i (block b: i in [64 b, 64 b + 64)); wave w sums the slices
// z = w, w + 4, ... in order, and the four wave sums are added in wave
// order: a fixed order for every launch.
__device__ __forceinline__ void sum_slices(const float *__restrict__ part, int nz, int64_t n, float *__restrict__ out,
                                           int64_t b)
{
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = b * 64 + lane;
    float sum = 0.f;
    if (i < n) {
#pragma unroll 4
        for (int z = w; z < nz; z += 4) sum += part[static_cast<int64_t>(z) * n + i];
    }
    red[w][lane] = sum;
    __syncthreads();
    if (w == 0 && i < n) out[i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// *out = sum of x[0 .. n): the block's first wave, lane-strided sums, then a
// fixed butterfly over the 64 lanes.
__device__ __forceinline__ void sum_wave(const float *__restrict__ x, int n, float *__restrict__ out)
{
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    float s = 0.f;
    for (int i = lane; i < n; i += 64) s += x[i];
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) *out = s;
}

// The output layer's backward pass in one launch: blocks [0, nb_back) the
// hidden-layer gradient (out_back), the next gx R blocks the weight-gradient
// partials (out_wgrad_part), the last block the batch loss (the sum of the
// per-block squared errors of k_out).
__global__ __launch_bounds__(256) void k_out_backward(OutBackArgs a)
{
    const int64_t b = blockIdx.x;
    if (b < a.nb_back) {
        out_back(a.dy, a.wo, a.width, a.Mrows, a.z, a.act, a.dz, a.dzb, a.dzbt, b);
    } else if (b < a.nb_back + static_cast<int64_t>(a.gx) * a.R) {
        const int q = static_cast<int>(b - a.nb_back);
        out_wgrad_part(a.dy, a.h, a.width, a.Mrows, a.pw, a.pb, q % a.gx, q / a.gx);
    } else {
        sum_wave(a.part, a.n_part, a.loss);
    }
}

// Block q of a pair of independent slice sums (sum_slices): the first sum's
// blocks, then the second's.
__device__ __forceinline__ void sum_pair(const SumPair &s, int64_t q)
{
    if (q < s.nba) sum_slices(s.a.part, s.a.nz, s.a.n, s.a.out, q);
    else sum_slices(s.b.part, s.b.nz, s.b.n, s.b.out, q - s.nba);
}

__global__ __launch_bounds__(256) void k_sum2(SumPair s) { sum_pair(s, blockIdx.x); }

// A split-K weight-gradient product (gemm_tile, float32 slices), the
// column-sum partials of the layer's output gradient (the bias gradient)
// and the slice sums of an earlier layer's gradients, which read none of
// this launch's outputs, in one launch: blocks [0, gx gy gz) the product,
// the next c.gx R the column sums, the rest the sums.
template <int NK>
__global__ __launch_bounds__(kGemmThreads) void k_wgrad_colsum(GemmArgs g, int gx, int gy, int gz, ColsumArgs c,
                                                               SumPair fold)
{
    const int64_t b = blockIdx.x, ng = static_cast<int64_t>(gx) * gy * gz, nc = static_cast<int64_t>(c.gx) * c.R;
    if (b < ng) {
        gemm_tile<kEpiF32, NK>(g, static_cast<int>(b % gx), static_cast<int>((b / gx) % gy),
                               static_cast<int>(b / (static_cast<int64_t>(gx) * gy)));
    } else if (b < ng + nc) {
        const int q = static_cast<int>(b - ng);
        colsum_part(c.x, c.rows, c.cols, c.part, q % c.gx, q / c.gx);
    } else {
        sum_pair(fold, b - ng - nc);
    }
}

// A product (no k split) and the slice sums of the previous layer's
// gradients, which it does not read, in one launch: blocks [0, gx gy) the
// product, the rest the sums.
template <int EPI, int NK, int TN>
__global__ __launch_bounds__(kGemmThreads) void k_gemm_fold(GemmArgs g, int gx, int gy, SumPair fold)
{
    const int64_t b = blockIdx.x, ng = static_cast<int64_t>(gx) * gy;
    if (b < ng) gemm_tile<EPI, NK, TN>(g, static_cast<int>(b % gx), static_cast<int>(b / gx), 0);
    else sum_pair(fold, b - ng);
}

// Fragment-major position of element (m, n) of a [rows][K] bf16 matrix
// (rows a multiple of 32, K of 16): 32 x 16 blocks, row block major, each
// block stored as the 64 lanes x 8 elements of a v_mfma_f32_32x32x16_bf16
// operand (lane m % 32 + 32 ((n / 8) % 2), element n % 8).
__device__ __forceinline__ int frag_index(int m, int n, int K)
{
    return ((((m >> 5) * (K >> 4) + (n >> 4)) * 64 + ((m & 31) + 32 * ((n >> 3) & 1))) << 3) + (n & 7);
}

// The bf16 copies of weight element j of layer l (value b): the plain copy,
// the transpose where one exists, the fragment-major copy where asked.
__device__ __forceinline__ void refresh_one(const RefreshTable &t, int l, int64_t j, uint16_t b)
{
    const int rows = t.rows[l], cols = t.cols[l];
    t.wb[t.woff[l] + j] = b;
    if (t.toff[l] >= 0) t.wt[t.toff[l] + static_cast<int64_t>(j % cols) * rows + j / cols] = b;
    if (t.frag[l]) t.wf[t.woff[l] + frag_index(static_cast<int>(j / cols), static_cast<int>(j % cols), cols)] = b;
}

// Adam over the parameters, then the bf16 copies of the updated weights
// (what k_refresh writes).  The step count *step (kept on the device so that
// a captured training epoch replays unchanged) was advanced at the start of
// this training step: the step number is t = *step, the learning rate
// lr_sched[*step - 1 - step0], the bias corrections 1 - b^t.
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t n, const float *__restrict__ lr_sched,
                       const int64_t *__restrict__ step, int64_t step0, float b1, float b2, float eps, RefreshTable rt)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = *step - 1;
    const float lr = lr_sched[s - step0];
    const float t = static_cast<float>(s + 1);
    const float bc1 = 1.0f - powf(b1, t), bc2 = 1.0f - powf(b2, t);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    for (int l = 0; l < rt.n_layers; ++l) {  // weights (not biases) get bf16 copies
        const int64_t j = i - rt.woff[l];
        if (j >= 0 && j < static_cast<int64_t>(rt.rows[l]) * rt.cols[l]) refresh_one(rt, l, j, to_bf16(wi));
    }
}

// bf16 copies of every weight matrix [rows][cols] and, where a transposed
// copy exists, of its transpose, and where asked a fragment-major copy;
// blockIdx.y = layer.
__global__ void k_refresh(RefreshTable t)
{
    const int l = blockIdx.y;
    const float *w = t.w + t.woff[l];
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
         i < static_cast<int64_t>(t.rows[l]) * t.cols[l]; i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        refresh_one(t, l, i, to_bf16(w[i]));
}

// ---------------------------------------------------------------- fused inference
// The whole network for 128 points per 256-thread block, width 256, two
// blocks per CU: the features and every hidden activation stay in one
// 128 x 256 bf16 LDS buffer, overwritten in place layer by layer, so HBM sees
// only the points and the outputs.  Each layer is computed transposed,
// z^T = W h^T: wave w owns output features [64 w, 64 w + 64) of all 128
// points, two 32-feature blocks of W (the A operand) times four 32-point
// blocks of h^T (the B operand), eight 32 x 32 MFMA accumulators.  Weights
// and activations are both stored fragment-major (frag_index: output
// features, resp. points, as rows), so every operand load is one contiguous
// 1 KB per wave.  The k loop is unrolled and its issue order pinned: per k
// step (LDS read, two MFMAs) per point block, the LDS reads running two
// ahead, then the weight loads for kPrefetch steps ahead (continuing into
// the next layer's first steps).  An accumulator register holds four
// consecutive features of one point: the epilogue adds the bias, applies the
// activation and stores them as one 8-byte LDS write.  The output layer (4
// features) is one more MFMA pass with W_out padded to 32 rows by zero lanes.
#ifndef SBR_FUSED_PB
#define SBR_FUSED_PB 4  // 32-point blocks per workgroup
#endif
#ifndef SBR_FUSED_OCC
#define SBR_FUSED_OCC 2  // workgroups per CU the register budget is set for
#endif
constexpr int kFusedPB = SBR_FUSED_PB, kFusedRows = 32 * kFusedPB, kFusedW = 256, kPrefetch = 4;

// One hidden layer's products for one wave: acc[fb][pb] += W block (fb0 +
// fb) times h^T block pb over NKS k steps, fully unrolled.  The B fragments
// (LDS) are read one step ahead; the weight ring wq is refilled kPrefetch
// steps ahead, from Wn (the next layer's weights) past the last steps.
template <int NKS>
__device__ __forceinline__ void fused_products(const bf16x8 *in, const bf16x8 *W, const bf16x8 *Wn, int fb0, int lane,
                                               bf16x8 (&wq)[kPrefetch][2], f32x16 (&acc)[2][kFusedPB])
{
    constexpr int nksn = kFusedW >> 4;  // k steps of every later layer
    bf16x8 bq[2][kFusedPB];
#pragma unroll
    for (int pb = 0; pb < kFusedPB; ++pb) bq[0][pb] = in[(pb * NKS) * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
        const int u = ks % kPrefetch;
        const bf16x8 a0 = wq[u][0], a1 = wq[u][1];
        if (ks + kPrefetch < NKS) {
            wq[u][0] = W[(fb0 * NKS + ks + kPrefetch) * 64 + lane];
            wq[u][1] = W[((fb0 + 1) * NKS + ks + kPrefetch) * 64 + lane];
        } else {
            wq[u][0] = Wn[(fb0 * nksn + ks + kPrefetch - NKS) * 64 + lane];
            wq[u][1] = Wn[((fb0 + 1) * nksn + ks + kPrefetch - NKS) * 64 + lane];
        }
        if (ks + 1 < NKS) {
#pragma unroll
            for (int pb = 0; pb < kFusedPB; ++pb) bq[(ks + 1) & 1][pb] = in[(pb * NKS + ks + 1) * 64 + lane];
        }
#pragma unroll
        for (int pb = 0; pb < kFusedPB; ++pb) {
            acc[0][pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, bq[ks & 1][pb], acc[0][pb], 0, 0, 0);
            acc[1][pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, bq[ks & 1][pb], acc[1][pb], 0, 0, 0);
        }
        // issue order of the step: (one LDS read, two MFMAs) x PB, then the two weight loads
#pragma unroll
        for (int pb = 0; pb < kFusedPB; ++pb) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
    }
}

template <int kAct>
__global__ __launch_bounds__(256, SBR_FUSED_OCC) void k_mlp_fused(FusedArgs f)
{
    __shared__ __attribute__((aligned(16))) uint16_t act[kFusedRows * kFusedW];
    __shared__ double xs[kFusedRows][3];
    __shared__ __attribute__((aligned(16))) float bsh[kMaxLayers - 1][kFusedW];  // hidden-layer biases
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, h = lane >> 5, c32 = lane & 31;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kFusedRows;
    const int K0 = 2 * f.n_ff;
    const int fb0 = 2 * wv;  // this wave's two 32-feature blocks
    // weight ring: slot u holds the k steps = u (mod kPrefetch) of the current
    // layer and, past its last steps, the first steps of the next layer; the
    // first layer's are in flight during the feature computation
    bf16x8 wq[kPrefetch][2];
    {
        const bf16x8 *W = reinterpret_cast<const bf16x8 *>(f.wf[0]);
        const int nks = K0 >> 4;
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u) {
            wq[u][0] = W[(fb0 * nks + u) * 64 + lane];
            wq[u][1] = W[((fb0 + 1) * nks + u) * 64 + lane];
        }
    }
    for (int i = tid; i < f.depth * kFusedW; i += 256) bsh[i / kFusedW][i % kFusedW] = f.b[i / kFusedW][i % kFusedW];
    if (tid < kFusedRows) {
        const int64_t m = row0 + tid;
        for (int c = 0; c < 3; ++c) xs[tid][c] = m < f.M ? norm_coord(f.pts + 3 * m, f.norm, c) : 0.0;
    }
    __syncthreads();
    {   // features -> act, width K0; n_ff divides 256, so each thread keeps one feature q
        const int q = tid % f.n_ff;
        const float Bq[3] = {f.Bff[3 * q], f.Bff[3 * q + 1], f.Bff[3 * q + 2]};
        for (int r = tid / f.n_ff; r < kFusedRows; r += 256 / f.n_ff) {
            uint16_t hs = 0, hc = 0;
            if (row0 + r < f.M) ff_pair(xs[r], Bq, hs, hc);
            act[frag_index(r, q, K0)] = hs;
            act[frag_index(r, f.n_ff + q, K0)] = hc;
        }
    }
    __syncthreads();
    const bf16x8 *in = reinterpret_cast<const bf16x8 *>(act);
    for (int l = 0; l < f.depth; ++l) {
        const bf16x8 *W = reinterpret_cast<const bf16x8 *>(f.wf[l]);
        // (past the last layer the ring reloads its own weights, unused)
        const bf16x8 *Wn = reinterpret_cast<const bf16x8 *>(f.wf[l + 1 < f.depth ? l + 1 : l]);
        // register q of a 32 x 32 accumulator holds feature 8 (q / 4) + 4 h +
        // q % 4 of its block; the bias is added in the epilogue
        f32x16 acc[2][kFusedPB];
#pragma unroll
        for (int fb = 0; fb < 2; ++fb)
#pragma unroll
            for (int pb = 0; pb < kFusedPB; ++pb) acc[fb][pb] = f32x16{};
        if (l == 0 && K0 == 128)
            fused_products<8>(in, W, Wn, fb0, lane, wq, acc);
        else
            fused_products<16>(in, W, Wn, fb0, lane, wq, acc);
        __syncthreads();  // every wave has read the layer input: overwrite it
#pragma unroll
        for (int fb = 0; fb < 2; ++fb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n0 = (fb0 + fb) * 32 + 8 * j + 4 * h;  // features n0 .. n0 + 3
                const float4 bn4 = *reinterpret_cast<const float4 *>(&bsh[l][n0]);
                const float bn[4] = {bn4.x, bn4.y, bn4.z, bn4.w};
#pragma unroll
                for (int pb = 0; pb < kFusedPB; ++pb) {
                    const f32x16 &c = acc[fb][pb];
                    const uint32_t lo = to_bf16x2(act_t<kAct>(c[4 * j] + bn[0]), act_t<kAct>(c[4 * j + 1] + bn[1]));
                    const uint32_t hi = to_bf16x2(act_t<kAct>(c[4 * j + 2] + bn[2]), act_t<kAct>(c[4 * j + 3] + bn[3]));
                    *reinterpret_cast<uint2 *>(act + frag_index(pb * 32 + c32, n0, kFusedW)) = make_uint2(lo, hi);
                }
            }
        __syncthreads();
    }
    // output layer: wave w takes the 32-point blocks w, w + 4, ...; lanes
    // 0..3 (and 32..35) of the A operand carry W_out's rows, the rest are zero
    const int nks = kFusedW >> 4;
    for (int pb = wv; pb < kFusedPB; pb += 4) {
        f32x16 y = f32x16{};
        for (int ks = 0; ks < nks; ++ks) {
            bf16x8 a = bf16x8{};
            if (c32 < 4) a = *reinterpret_cast<const bf16x8 *>(f.wo + c32 * kFusedW + ks * 16 + 8 * h);
            const bf16x8 b = in[(pb * nks + ks) * 64 + lane];
            y = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, y, 0, 0, 0);
        }
        // rows 0..3 of the result (outputs) sit in registers 0..3 of lanes 0..31
        const int64_t m = row0 + pb * 32 + c32;
        if (h == 0 && m < f.M) {
            for (int o = 0; o < 4; ++o) f.A[4 * m + o] = f.scale * (y[o] + f.bo[o]);
        }
    }
}

// ---------------------------------------------------------------- grid fill
// Points of an angle x frequency grid: pts[a * nf + f] = (theta_a, phi_a, f).
__global__ void k_grid_pts(const double *__restrict__ th, const double *__restrict__ ph, const double *__restrict__ fr,
                           int64_t na, int nf, double *__restrict__ pts)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= na * nf) return;
    const int64_t a = i / nf;
    const int f = static_cast<int>(i % nf);
    pts[3 * i] = th[a];
    pts[3 * i + 1] = ph[a];
    pts[3 * i + 2] = fr[f];
}

__device__ __forceinline__ double sig_db(double re, double im)
{
    const double s = 4.0 * 3.14159265358979323846 * (re * re + im * im);
    return s > 0.0 ? 10.0 * log10(s) : -400.0;
}

// Largest co-polar sigma (dBsm) of the SBR probe results [n][2][2] complex.
__global__ void k_probe_max(const double *__restrict__ A, int64_t n, double *__restrict__ out)
{
    __shared__ double red[256];
    double m = -400.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double *q = A + 8 * i;
        m = fmax(m, fmax(sig_db(q[0], q[1]), sig_db(q[6], q[7])));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// One thread per tile (ta, tf): largest |sigma_sur - sigma_sbr| (dB) over the
// tile's probes (per_tile consecutive probe frequencies of angle tile ta),
// both co-polar channels, counting only probes whose SBR sigma is at least
// smax - floor_db; flag = 1 when it exceeds tol_db.
__global__ void k_probe_check(const double *__restrict__ A_sbr, const double *__restrict__ A_sur, int64_t n_ta,
                              int n_tf, int per_tile, const double *__restrict__ smax, double floor_db, double tol_db,
                              uint8_t *__restrict__ flag, double *__restrict__ err)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_ta * n_tf) return;
    const int64_t ta = t / n_tf;
    const int tf = static_cast<int>(t % n_tf);
    const double lim = *smax - floor_db;
    double e = 0.0;
    for (int q = 0; q < per_tile; ++q) {
        const int64_t row = ta * static_cast<int64_t>(n_tf) * per_tile + static_cast<int64_t>(tf) * per_tile + q;
        const double *s = A_sbr + 8 * row;
        const double *u = A_sur + 4 * row;
        const double sh = sig_db(s[0], s[1]), sv = sig_db(s[6], s[7]);
        if (sh >= lim) e = fmax(e, fabs(sig_db(u[0], u[1]) - sh));
        if (sv >= lim) e = fmax(e, fabs(sig_db(u[2], u[3]) - sv));
    }
    err[t] = e;
    flag[t] = e > tol_db ? 1 : 0;
}

// SBR rows [n][2][2] complex -> grid entries dst[r] of [.][2] complex (HH, VV).
__global__ void k_scatter_copol(const double *__restrict__ A, const int64_t *__restrict__ dst, int64_t n,
                                double *__restrict__ out)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n || dst[r] < 0) return;  // dst < 0: a row computed but not wanted
    const double *q = A + 8 * r;
    double *o = out + 4 * dst[r];
    o[0] = q[0];
    o[1] = q[1];
    o[2] = q[6];
    o[3] = q[7];
}

inline unsigned nblk(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

int launch_gemm(hipStream_t s, int epi, const GemmArgs &g)
{
    if (g.M % kTileM || g.N % kTileN || g.K % 16 || g.K <= 0)
        return fail(SBR_ERR_INVALID_ARG, "MLP product: shape not a multiple of the 64 x 128 x 16 tile");
    if (g.ksplit < 1 || (g.K / g.ksplit) % 16 || g.K % g.ksplit || (g.ksplit > 1 && epi != kEpiF32))
        return fail(SBR_ERR_INVALID_ARG, "MLP product: bad k split");
    if (g.htout && (g.ldht % 4 || reinterpret_cast<uintptr_t>(g.htout) % 8))
        return fail(SBR_ERR_INVALID_ARG, "MLP product: transposed output not 8-byte aligned");
    // 64 x 64 tiles when 64 x 128 ones would leave CUs idle
    const bool narrow = (g.M / kTileM) * (g.N / kTileN) * g.ksplit < 256;
    dim3 grid(g.M / kTileM, g.N / (narrow ? 64 : kTileN), g.ksplit);
    const int nk = g.K / g.ksplit / 16;
    auto go = [&](auto epi_c) {
        constexpr int E = decltype(epi_c)::value;
        if (narrow) {
            if (nk == 8) k_gemm<E, 8, 64><<<grid, kGemmThreads, 0, s>>>(g);
            else if (nk == 16) k_gemm<E, 16, 64><<<grid, kGemmThreads, 0, s>>>(g);
            else k_gemm<E, 0, 64><<<grid, kGemmThreads, 0, s>>>(g);
        } else {
            if (nk == 8) k_gemm<E, 8, kTileN><<<grid, kGemmThreads, 0, s>>>(g);
            else if (nk == 16) k_gemm<E, 16, kTileN><<<grid, kGemmThreads, 0, s>>>(g);
            else k_gemm<E, 0, kTileN><<<grid, kGemmThreads, 0, s>>>(g);
        }
    };
    if (epi == kEpiHidden) go(std::integral_constant<int, kEpiHidden>{});
    else if (epi == kEpiDz) go(std::integral_constant<int, kEpiDz>{});
    else go(std::integral_constant<int, kEpiF32>{});
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_embed(hipStream_t s, const double *pts, int64_t M, int64_t Mpad, const MlpNorm &nm, const float *Bff,
                 int n_ff, uint16_t *h0, uint16_t *h0t)
{
    k_embed<<<nblk(Mpad * n_ff, 256), 256, 0, s>>>(pts, M, Mpad, nm, Bff, n_ff, h0, h0t);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_out(hipStream_t s, const uint16_t *h, int width, const uint16_t *wo, const float *bo, int64_t M,
               int64_t Mrows, int mode, double scale, double *A, const float *tgt, float *dy, float *partial)
{
    k_out<<<nblk(Mrows, 16), 256, 0, s>>>(h, width, wo, bo, M, Mrows, mode, scale, A, tgt, dy, partial);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_embed_batch(hipStream_t s, const double *pts, const double *tc, const int32_t *idx, int64_t count,
                       int64_t Mpad, const MlpNorm &nm, const float *Bff, int n_ff, double inv_scale, uint16_t *h0,
                       uint16_t *h0t, float *tb, int64_t *bump)
{
    k_embed_batch<<<nblk(Mpad * n_ff, 256), 256, 0, s>>>(pts, tc, idx, count, Mpad, nm, Bff, n_ff, inv_scale, h0, h0t, tb,
                                                          bump);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

SumPair sum_pair_of(const SumJob &a, const SumJob &b)
{
    return SumPair{a, b, static_cast<int64_t>(nblk(a.n, 64)), static_cast<int64_t>(nblk(b.n, 64))};
}

int launch_out_backward(hipStream_t s, const OutBackIn &in, float *gw, float *gb, float *scratch, SumPair *pending)
{
    const int R = static_cast<int>((in.Mrows + 63) / 64);
    if (in.Mrows % 64) return fail(SBR_ERR_INVALID_ARG, "MLP output backward: rows not a multiple of 64");
    OutBackArgs a{};
    static_cast<OutBackIn &>(a) = in;
    a.pw = scratch;
    a.pb = scratch + static_cast<int64_t>(R) * 4 * in.width;
    a.nb_back = nblk((in.Mrows / 4) * in.width, 256);
    a.gx = (in.width + 63) / 64;
    a.R = R;
    k_out_backward<<<static_cast<unsigned>(a.nb_back + static_cast<int64_t>(a.gx) * R + 1), 256, 0, s>>>(a);
    *pending = sum_pair_of(SumJob{a.pw, R, 4 * static_cast<int64_t>(in.width), gw}, SumJob{a.pb, R, 4, gb});
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_wgrad_colsum(hipStream_t s, const GemmArgs &g, const float *dz, int64_t rows, int cols, float *colpart,
                        float *gw, float *gb, const SumPair &fold, SumPair *pending)
{
    if (g.M % kTileM || g.N % kTileN || g.K % 16 || g.K <= 0 || g.ksplit < 1 || g.K % g.ksplit ||
        (g.K / g.ksplit) % 16 || !g.fout)
        return fail(SBR_ERR_INVALID_ARG, "MLP weight gradient: shape not a multiple of the tile");
    const int gx = g.M / kTileM, gy = g.N / kTileN, gz = g.ksplit;
    const int R = static_cast<int>((rows + 63) / 64);
    ColsumArgs c{dz, rows, cols, colpart, (cols + 63) / 64, R};
    const unsigned nb = static_cast<unsigned>(static_cast<int64_t>(gx) * gy * gz + static_cast<int64_t>(c.gx) * R +
                                              fold.nba + fold.nbb);
    const int nk = g.K / g.ksplit / 16;
    if (nk == 8) k_wgrad_colsum<8><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, gz, c, fold);
    else if (nk == 16) k_wgrad_colsum<16><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, gz, c, fold);
    else k_wgrad_colsum<0><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, gz, c, fold);
    *pending = sum_pair_of(SumJob{g.fout, g.ksplit, static_cast<int64_t>(g.M) * g.N, gw}, SumJob{colpart, R, cols, gb});
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_gemm_fold(hipStream_t s, int epi, const GemmArgs &g, const SumPair &fold)
{
    if (g.M % kTileM || g.N % kTileN || g.K % 16 || g.K <= 0 || g.ksplit != 1 || epi == kEpiF32)
        return fail(SBR_ERR_INVALID_ARG, "MLP product with sums: shape not a multiple of the tile");
    if (g.htout && (g.ldht % 4 || reinterpret_cast<uintptr_t>(g.htout) % 8))
        return fail(SBR_ERR_INVALID_ARG, "MLP product: transposed output not 8-byte aligned");
    // 64 x 64 tiles when 64 x 128 ones would leave CUs idle (as launch_gemm)
    const bool narrow = (g.M / kTileM) * (g.N / kTileN) < 256;
    const int gx = g.M / kTileM, gy = g.N / (narrow ? 64 : kTileN);
    const unsigned nb = static_cast<unsigned>(static_cast<int64_t>(gx) * gy + fold.nba + fold.nbb);
    const int nk = g.K / 16;
    auto go = [&](auto epi_c) {
        constexpr int E = decltype(epi_c)::value;
        if (narrow) {
            if (nk == 8) k_gemm_fold<E, 8, 64><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, fold);
            else if (nk == 16) k_gemm_fold<E, 16, 64><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, fold);
            else k_gemm_fold<E, 0, 64><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, fold);
        } else {
            if (nk == 8) k_gemm_fold<E, 8, kTileN><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, fold);
            else if (nk == 16) k_gemm_fold<E, 16, kTileN><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, fold);
            else k_gemm_fold<E, 0, kTileN><<<nb, kGemmThreads, 0, s>>>(g, gx, gy, fold);
        }
    };
    if (epi == kEpiHidden) go(std::integral_constant<int, kEpiHidden>{});
    else go(std::integral_constant<int, kEpiDz>{});
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_sum_pair(hipStream_t s, const SumPair &p)
{
    if (p.nba + p.nbb > 0) k_sum2<<<static_cast<unsigned>(p.nba + p.nbb), 256, 0, s>>>(p);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_adam(hipStream_t s, float *w, float *m, float *v, const float *g, int64_t n, const float *lr_sched,
                const int64_t *step, int64_t step0, float b1, float b2, float eps, const RefreshTable &rt)
{
    if (rt.n_layers < 1 || rt.n_layers > kMaxLayers) return fail(SBR_ERR_INVALID_ARG, "adam: layer count");
    k_adam<<<nblk(n, 256), 256, 0, s>>>(w, m, v, g, n, lr_sched, step, step0, b1, b2, eps, rt);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_refresh(hipStream_t s, const RefreshTable &t)
{
    if (t.n_layers < 1 || t.n_layers > kMaxLayers) return fail(SBR_ERR_INVALID_ARG, "refresh: layer count");
    dim3 grid(64, t.n_layers);
    k_refresh<<<grid, 256, 0, s>>>(t);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_grid_pts(hipStream_t s, const double *th, const double *ph, const double *fr, int64_t na, int nf,
                    double *pts)
{
    k_grid_pts<<<nblk(na * nf, 256), 256, 0, s>>>(th, ph, fr, na, nf, pts);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_probe_check(hipStream_t s, const double *A_sbr, const double *A_sur, int64_t n_ta, int n_tf, int per_tile,
                       double *smax, double floor_db, double tol_db, uint8_t *flag, double *err)
{
    k_probe_max<<<1, 256, 0, s>>>(A_sbr, n_ta * n_tf * per_tile, smax);
    k_probe_check<<<nblk(n_ta * n_tf, 256), 256, 0, s>>>(A_sbr, A_sur, n_ta, n_tf, per_tile, smax, floor_db, tol_db,
                                                       flag, err);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_scatter_copol(hipStream_t s, const double *A, const int64_t *dst, int64_t n, double *out)
{
    if (n <= 0) return SBR_OK;
    k_scatter_copol<<<nblk(n, 256), 256, 0, s>>>(A, dst, n, out);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

// (k_mlp_fused unrolls the first layer for 8 or 16 k steps)
bool fused_ok(int n_ff, int width, int depth)
{
    return width == kFusedW && (n_ff == 64 || n_ff == 128) && depth >= 1 && depth <= kMaxLayers - 1;
}

int launch_mlp_fused(hipStream_t s, const FusedArgs &f)
{
    if (f.M <= 0) return SBR_OK;
    if (f.act == kActSilu)
        k_mlp_fused<kActSilu><<<nblk(f.M, kFusedRows), 256, 0, s>>>(f);
    else
        k_mlp_fused<kActRelu><<<nblk(f.M, kFusedRows), 256, 0, s>>>(f);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

}  // namespace sbr
