// Ray-tube physical-optics sum and RCS (Eq. po_sum; Eqs. em5-em6; Sec. 4
// trace-integrate paragraph: the integrate stage is a reduction over the
// valid hit records).
//
// Every valid record contributes, per frequency f and (receive p, transmit q)
// pair, a_pq = -j (k_f dA / 2 pi) w_pq exp(-j k_f D):
//   PAPER:  w = (n0 . -k) (-1)^(N+1) on the co-polar pairs (Gamma = -1);
//   VECTOR: w_pq = (J_q . p_hat) / c_L, J_q = d (n.e_q) - e_q (n.d), n the
//           facing normal at the last hit, c_L = max(-n.d, 1e-3).
// The kernel accumulates sum w sin(kD) and sum w cos(kD); the constant
// -(k dA / 2 pi) is applied in the finalize step.
//
// Numerics: the phase k_f * D is formed and reduced modulo 2 pi in float64
// (k D reaches 1e3-1e4 rad), sin/cos and w are float32.  Each term is
// converted to a 64-bit fixed-point integer (unit 2^-32) and summed as an
// integer, so the per-block partials do not depend on the order in which the
// trace stage appended its records: results are bitwise reproducible without
// any float atomics.  The wave reduction uses DPP row permutations (quad
// swaps, half-row and row mirrors) and four lane reads; waves are combined
// through LDS into one partial per block; the finalize kernel sums the
// partials of an angle in fixed block order in float64.
#include <cmath>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

constexpr int kPoThreads = 256;
constexpr int kFT = 2;  // frequencies per pass over a block's records

struct PoP {
    Records rec;
    const uint32_t *rec_cnt;
    int cnt_stride;
    const int64_t *rec_base;
    const float4 *nrm_id;
    int chunks;
    int mode;
    const double *kf;
    int n_freq;
    const double *basis;
    long long *partial;
};

template <int CTRL>
__device__ __forceinline__ long long dpp64(long long x)
{
    const int lo = static_cast<int>(x);
    const int hi = static_cast<int>(x >> 32);
    const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
    const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
    return static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(h2)) << 32) |
                                  static_cast<unsigned>(l2));
}

__device__ __forceinline__ long long readlane64(long long x, int lane)
{
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(x), lane);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(x >> 32), lane);
    return static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                  static_cast<unsigned>(lo));
}

// Sum over the 64 lanes (all lanes must be active); result is wave-uniform.
__device__ __forceinline__ long long wave_sum64(long long x)
{
    x += dpp64<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp64<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp64<0x141>(x);  // row_half_mirror
    x += dpp64<0x140>(x);  // row_mirror: every lane holds its row's sum
    return readlane64(x, 0) + readlane64(x, 16) + readlane64(x, 32) + readlane64(x, 48);
}

// round(x * 2^32) as a 64-bit integer for |x| < 2^19, via the float64
// rounding of x * 2^32 + 1.5 * 2^52.
__device__ __forceinline__ long long fix32(float x)
{
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    const double y = __builtin_fma(static_cast<double>(x), 4294967296.0, magic);
    return __double_as_longlong(y) - __double_as_longlong(magic);
}

__device__ __forceinline__ void weights(const PoP &p, int a, const float4 r0, const float4 r1, const float4 r2,
                                        float w[4])
{
    const int meta = __float_as_int(r2.w);
    const int N = meta & 255;
    const int flags = meta >> 8;
    w[0] = w[1] = w[2] = w[3] = 0.0f;
    if (!(flags & SBR_REC_VALID)) return;
    const double *B = p.basis + 9 * a;
    if (p.mode == SBR_MODE_PAPER) {
        const float4 n0 = p.nrm_id[__float_as_int(r1.w)];
        const float c0 = fabsf((n0.x * static_cast<float>(B[0]) + n0.y * static_cast<float>(B[1])) +
                               n0.z * static_cast<float>(B[2]));
        const float s = (N & 1) ? c0 : -c0;
        w[0] = s;
        w[3] = s;
        return;
    }
    float4 n = p.nrm_id[__float_as_int(r0.w)];
    if (flags & SBR_REC_BACK_LAST) {
        n.x = -n.x;
        n.y = -n.y;
        n.z = -n.z;
    }
    const float ndl = (n.x * r0.x + n.y * r0.y) + n.z * r0.z;
    const float c = fmaxf(-ndl, 1e-3f);
    const float ic = 1.0f / c;
    const float thx = static_cast<float>(B[3]), thy = static_cast<float>(B[4]), thz = static_cast<float>(B[5]);
    const float phx = static_cast<float>(B[6]), phy = static_cast<float>(B[7]), phz = static_cast<float>(B[8]);
    // q = 0: H (r1.xyz), q = 1: V (r2.xyz); p = 0: H (phi_hat), p = 1: V (theta_hat)
    for (int q = 0; q < 2; ++q) {
        const float ex = q ? r2.x : r1.x, ey = q ? r2.y : r1.y, ez = q ? r2.z : r1.z;
        const float ne = (n.x * ex + n.y * ey) + n.z * ez;
        const float jx = r0.x * ne - ex * ndl, jy = r0.y * ne - ey * ndl, jz = r0.z * ne - ez * ndl;
        w[0 * 2 + q] = ((jx * phx + jy * phy) + jz * phz) * ic;
        w[1 * 2 + q] = ((jx * thx + jy * thy) + jz * thz) * ic;
    }
}

__global__ __launch_bounds__(kPoThreads) void k_po(PoP p)
{
    __shared__ long long red[kPoThreads / 64][kFT * 8];
    const int a = blockIdx.y, c = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t cnt = p.rec_cnt[static_cast<int64_t>(a) * p.cnt_stride];
    const int64_t base = p.rec_base[a];
    const int64_t r0i = static_cast<int64_t>(c) * kPoRecsPerBlock;
    long long *out = p.partial + ((static_cast<int64_t>(a) * p.chunks + c) * p.n_freq) * 8;
    if (r0i >= cnt) return;  // the finalize step reads only the chunks that hold records
    const int64_t r1i = min(r0i + kPoRecsPerBlock, cnt);
    const double two_pi_hi = 6.283185307179586;       // fl64(2 pi)
    const double two_pi_lo = 2.4492935982947064e-16;  // 2 pi - fl64(2 pi)
    const double inv_two_pi = 0.15915494309189535;
    for (int f0 = 0; f0 < p.n_freq; f0 += kFT) {
        long long acc[kFT][8];
        for (int ft = 0; ft < kFT; ++ft)
            for (int e = 0; e < 8; ++e) acc[ft][e] = 0;
        for (int64_t e = base + r0i + tid; e < base + r1i; e += kPoThreads) {
            const float4 q2 = p.rec.r2[e];
            if (!((__float_as_int(q2.w) >> 8) & SBR_REC_VALID)) continue;  // no hit (or dropped): no term
            const float4 q0 = p.rec.r0[e], q1 = p.rec.r1[e];
            const double D = p.rec.D[e];
            float w[4];
            weights(p, a, q0, q1, q2, w);
            for (int ft = 0; ft < kFT; ++ft) {
                const int f = f0 + ft;
                if (f >= p.n_freq) break;
                const double ph = p.kf[f] * D;
                const double nturn = rint(ph * inv_two_pi);
                const double red_ph = __builtin_fma(-nturn, two_pi_lo, __builtin_fma(-nturn, two_pi_hi, ph));
                float s, co;
                sincosf(static_cast<float>(red_ph), &s, &co);
                for (int k = 0; k < 4; ++k) {
                    acc[ft][2 * k] += fix32(w[k] * s);
                    acc[ft][2 * k + 1] += fix32(w[k] * co);
                }
            }
        }
        for (int ft = 0; ft < kFT; ++ft)
            for (int k = 0; k < 8; ++k) {
                const long long s = wave_sum64(acc[ft][k]);
                if (lane == 0) red[wv][ft * 8 + k] = s;
            }
        __syncthreads();
        if (tid < kFT * 8) {
            const int ft = tid / 8, k = tid % 8;
            if (f0 + ft < p.n_freq) {
                long long s = 0;
                for (int x = 0; x < kPoThreads / 64; ++x) s += red[x][tid];
                out[(f0 + ft) * 8 + k] = s;
            }
        }
        __syncthreads();
    }
}

// One thread per (angle, frequency): fixed-order sum of the block partials.
__global__ void k_po_final(const long long *__restrict__ partial, const uint32_t *__restrict__ rec_cnt, int cnt_stride,
                           int n_angles, int chunks, int n_freq, const double *__restrict__ kf, double dA,
                           double *__restrict__ A_out, double *__restrict__ sigma)
{
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(n_angles) * n_freq) return;
    const int a = static_cast<int>(idx / n_freq), f = static_cast<int>(idx % n_freq);
    const int64_t nch = (static_cast<int64_t>(rec_cnt[static_cast<int64_t>(a) * cnt_stride]) + kPoRecsPerBlock - 1) /
                        kPoRecsPerBlock;
    double S[8];
    for (int e = 0; e < 8; ++e) S[e] = 0.0;
    for (int64_t c = 0; c < nch; ++c) {
        const long long *q = partial + ((static_cast<int64_t>(a) * chunks + c) * n_freq + f) * 8;
        for (int e = 0; e < 8; ++e) S[e] += static_cast<double>(q[e]);
    }
    const double C = -(kf[f] * dA / (2.0 * kPi)) * 2.3283064365386963e-10;  // 2^-32
    double *A = A_out + idx * 8;
    for (int k = 0; k < 4; ++k) {
        const double re = C * S[2 * k], im = C * S[2 * k + 1];
        A[2 * k] = re;
        A[2 * k + 1] = im;
        if (sigma) {
            const double sg = 4.0 * kPi * (re * re + im * im);
            sigma[idx * 4 + k] = sg > 0.0 ? 10.0 * log10(sg) : -400.0;
        }
    }
}

__global__ void k_pack(sbr_hits h, int64_t n, Records rec, uint32_t *cnt)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool in = e < n;
    const int fl = in ? h.flags[e] : 0;
    const bool want = in && (fl & SBR_REC_VALID);
    const uint64_t m = __ballot(want);
    uint32_t base = 0;
    if (m) {
        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
        if ((threadIdx.x & 63) == leader) base = atomicAdd(cnt, static_cast<uint32_t>(__popcll(m)));
        base = __shfl(base, leader);
    }
    if (!want) return;
    const uint32_t pos = base + __popcll(m & ((1ull << (threadIdx.x & 63)) - 1ull));
    rec.r0[pos] = make_float4(h.d_last[3 * e], h.d_last[3 * e + 1], h.d_last[3 * e + 2], __int_as_float(h.tri_last[e]));
    rec.r1[pos] = make_float4(h.eH_last[3 * e], h.eH_last[3 * e + 1], h.eH_last[3 * e + 2],
                              __int_as_float(h.tri_first[e]));
    rec.r2[pos] = make_float4(h.eV_last[3 * e], h.eV_last[3 * e + 1], h.eV_last[3 * e + 2],
                              __int_as_float((h.n_bounce[e] & 255) | (fl << 8)));
    rec.D[pos] = h.D[e];
}

}  // namespace

int launch_po(hipStream_t s, const PoArgs &a)
{
    PoP p;
    p.rec = a.rec;
    p.rec_cnt = a.rec_cnt;
    p.cnt_stride = a.cnt_stride;
    p.rec_base = a.rec_base;
    p.nrm_id = a.bvh->nrm_id;
    p.chunks = a.chunks;
    p.mode = a.mode;
    p.kf = a.kf;
    p.n_freq = a.n_freq;
    p.basis = a.basis;
    p.partial = a.partial;
    dim3 grid(a.chunks, a.n_angles);
    k_po<<<grid, kPoThreads, 0, s>>>(p);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_po_finalize(hipStream_t s, const PoArgs &a, double dA, double *A_out, double *sigma_out)
{
    const int64_t n = static_cast<int64_t>(a.n_angles) * a.n_freq;
    k_po_final<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(a.partial, a.rec_cnt, a.cnt_stride, a.n_angles, a.chunks,
                                                                      a.n_freq, a.kf, dA, A_out, sigma_out);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_pack_hits(hipStream_t s, const sbr_hits *h, int64_t n, Records rec, uint32_t *cnt)
{
    k_pack<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(*h, n, rec, cnt);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

}  // namespace sbr
