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
// (k D reaches 1e3-1e4 rad); its sine and cosine and the weights w are
// float64 (from the float32 records).  Float32 sine and cosine of the phase
// are not enough: on weak, strongly cancelling returns their rounding of
// ~1e-7 per term reaches 1e-4 of the result.  For evenly spaced wavenumbers
// the phasor of the next frequency is the previous one turned by dk D.
// A thread sums its own records (the slots tid, tid + 256, ... of its block,
// in that order) in float64; each thread sum is converted to a 64-bit
// fixed-point integer (unit 2^-32) and reduced as an integer.  The slots of
// a ray are fixed by its position in the aperture, so the result is bitwise
// reproducible across runs, schedules and launch parameters without any
// float atomics.  The wave reduction uses DPP row permutations (quad swaps,
// half-row and row mirrors) and four lane reads; waves are combined through
// LDS into one partial per block; the finalize kernel sums the partials of
// an angle in fixed block order in float64.
#include <cmath>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

constexpr int kPoThreads = 256;

struct PoP {
    Records rec;
    const PoAngle *ang;
    int n_angles;
    const float4 *nrm_id;
    int mode;
    const double *kf;
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

// sin and cos of x in [-pi, pi] in float64: x = q pi/2 + r with q = rint(x 2/pi)
// (pi/2 as a two-term sum, so r is exact to ~1e-17), |r| <= pi/4, then the
// Taylor polynomials of sin (through r^17) and cos (through r^18) in Horner
// form (truncation below 1e-18 on |r| <= pi/4), and the quadrant symmetries
// of sin and cos.  Absolute error about 1e-16.
__device__ __forceinline__ void sincos_pi(double x, double &so, double &co)
{
    const double pio2_hi = 1.5707963267948966;     // fl64(pi / 2)
    const double pio2_lo = 6.123233995736766e-17;  // pi / 2 - fl64(pi / 2)
    const double q = rint(x * 0.6366197723675814);
    double r = __builtin_fma(-q, pio2_hi, x);
    r = __builtin_fma(-q, pio2_lo, r);
    const double z = r * r;
    // (-1)^i / (2i + 1)!, i = 1..8 and (-1)^i / (2i)!, i = 1..9
    double ps = 1.0 / 355687428096000.0;
    ps = __builtin_fma(ps, z, -1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, z, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, z, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, z, 1.0 / 362880.0);
    ps = __builtin_fma(ps, z, -1.0 / 5040.0);
    ps = __builtin_fma(ps, z, 1.0 / 120.0);
    ps = __builtin_fma(ps, z, -1.0 / 6.0);
    const double sn = __builtin_fma(r * z, ps, r);
    double pc = -1.0 / 6402373705728000.0;
    pc = __builtin_fma(pc, z, 1.0 / 20922789888000.0);
    pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);
    pc = __builtin_fma(pc, z, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, z, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, z, 1.0 / 40320.0);
    pc = __builtin_fma(pc, z, -1.0 / 720.0);
    pc = __builtin_fma(pc, z, 1.0 / 24.0);
    pc = __builtin_fma(pc, z, -0.5);
    const double cs = __builtin_fma(z, pc, 1.0);
    const int qi = static_cast<int>(q) & 3;  // two's complement: -1 -> 3, -2 -> 2
    so = qi == 0 ? sn : qi == 1 ? cs : qi == 2 ? -sn : -cs;
    co = qi == 0 ? cs : qi == 1 ? -sn : qi == 2 ? -cs : sn;
}

// round(x * 2^32) as a 64-bit integer for |x| < 2^19, via the float64
// rounding of x * 2^32 + 1.5 * 2^52.
__device__ __forceinline__ long long fix32(double x)
{
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    const double y = __builtin_fma(x, 4294967296.0, magic);
    return __double_as_longlong(y) - __double_as_longlong(magic);
}

// Per-record weights w[p * 2 + q] in float64 from the float32 record fields:
// the cross-polar weights of VECTOR mode are differences of nearly equal
// products, and their float32 rounding, identical for the many rays of a flat
// facet, would add up coherently.
__device__ __forceinline__ void weights(const PoP &p, const double *B, const float4 r0, const float4 r1,
                                        const float4 r2, double w[4])
{
    const int meta = __float_as_int(r2.w);
    const int N = meta & 255;
    const int flags = meta >> 8;
    w[0] = w[1] = w[2] = w[3] = 0.0;
    if (!(flags & SBR_REC_VALID)) return;
    if (p.mode == SBR_MODE_PAPER) {
        const float4 n0 = p.nrm_id[__float_as_int(r1.w)];
        const double c0 = fabs((static_cast<double>(n0.x) * B[0] + static_cast<double>(n0.y) * B[1]) +
                               static_cast<double>(n0.z) * B[2]);
        const double s = (N & 1) ? c0 : -c0;
        w[0] = s;
        w[3] = s;
        return;
    }
    const float4 n32 = p.nrm_id[__float_as_int(r0.w)];
    const double sg = (flags & SBR_REC_BACK_LAST) ? -1.0 : 1.0;
    const double nx = sg * n32.x, ny = sg * n32.y, nz = sg * n32.z;
    const double dx = r0.x, dy = r0.y, dz = r0.z;
    const double ndl = (nx * dx + ny * dy) + nz * dz;
    const double c = fmax(-ndl, 1e-3);
    const double ic = 1.0 / c;
    // q = 0: H (r1.xyz), q = 1: V (r2.xyz); p = 0: H (phi_hat = B[6..8]), p = 1: V (theta_hat = B[3..5])
    for (int q = 0; q < 2; ++q) {
        const double ex = q ? r2.x : r1.x, ey = q ? r2.y : r1.y, ez = q ? r2.z : r1.z;
        const double ne = (nx * ex + ny * ey) + nz * ez;
        const double jx = dx * ne - ex * ndl, jy = dy * ne - ey * ndl, jz = dz * ne - ez * ndl;
        w[0 * 2 + q] = ((jx * B[6] + jy * B[7]) + jz * B[8]) * ic;
        w[1 * 2 + q] = ((jx * B[3] + jy * B[4]) + jz * B[5]) * ic;
    }
}

// Block u of the launch: records [c * kPoRecsPerBlock, (c + 1) * kPoRecsPerBlock)
// of angle a, where a is the angle whose blocks hold u and c = u - unit_base.
template <int kFT>  // frequencies per pass over a block's records
__global__ __launch_bounds__(kPoThreads) void k_po(PoP p)
{
    __shared__ long long red[kPoThreads / 64][kFT * 8];
    const int64_t u = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int lo = 0, hi = p.n_angles;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (p.ang[mid].unit_base <= u) lo = mid;
        else hi = mid;
    }
    const PoAngle &A = p.ang[lo];
    const int64_t c = u - A.unit_base;
    const int nf = A.n_f;
    const double *kf = p.kf + A.kf_off;
    long long *out = p.partial + (A.part_base + c * nf) * 8;
    const int64_t r0i = c * kPoRecsPerBlock;
    const int64_t r1i = min(r0i + kPoRecsPerBlock, A.rec_cnt);
    const double two_pi_hi = 6.283185307179586;       // fl64(2 pi)
    const double two_pi_lo = 2.4492935982947064e-16;  // 2 pi - fl64(2 pi)
    const double inv_two_pi = 0.15915494309189535;
    const bool uniform = A.dk != 0.0;
    for (int f0 = 0; f0 < nf; f0 += kFT) {
        // each thread sums its records (a fixed subset, in a fixed order) in
        // float64; the per-thread sums become fixed point before the exact
        // integer reduction over threads, waves and blocks
        double acc[kFT][8];
        for (int ft = 0; ft < kFT; ++ft)
            for (int e = 0; e < 8; ++e) acc[ft][e] = 0.0;
        for (int64_t e = A.rec_base + r0i + tid; e < A.rec_base + r1i; e += kPoThreads) {
            const float4 q2 = p.rec.r2[e];
            if (!((__float_as_int(q2.w) >> 8) & SBR_REC_VALID)) continue;  // no hit (or dropped): no term
            const float4 q0 = p.rec.r0[e], q1 = p.rec.r1[e];
            const double D = p.rec.D[e];
            double w[4];
            weights(p, A.basis, q0, q1, q2, w);
            double sd, cd, rs = 0.0, rc = 1.0;
            {
                const double ph = kf[f0] * D;
                const double nturn = rint(ph * inv_two_pi);
                sincos_pi(__builtin_fma(-nturn, two_pi_lo, __builtin_fma(-nturn, two_pi_hi, ph)), sd, cd);
            }
            if (uniform) {  // evenly spaced wavenumbers: each step turns the phasor by dk D
                const double ph = A.dk * D;
                const double nturn = rint(ph * inv_two_pi);
                sincos_pi(__builtin_fma(-nturn, two_pi_lo, __builtin_fma(-nturn, two_pi_hi, ph)), rs, rc);
            }
#pragma unroll
            for (int ft = 0; ft < kFT; ++ft) {
                const int f = f0 + ft;
                if (f >= nf) break;
                if (ft > 0) {
                    if (uniform) {
                        const double s2 = __builtin_fma(sd, rc, cd * rs);
                        cd = __builtin_fma(cd, rc, -(sd * rs));
                        sd = s2;
                    } else {
                        const double ph = kf[f] * D;
                        const double nturn = rint(ph * inv_two_pi);
                        sincos_pi(__builtin_fma(-nturn, two_pi_lo, __builtin_fma(-nturn, two_pi_hi, ph)), sd, cd);
                    }
                }
                for (int k = 0; k < 4; ++k) {
                    acc[ft][2 * k] = __builtin_fma(w[k], sd, acc[ft][2 * k]);
                    acc[ft][2 * k + 1] = __builtin_fma(w[k], cd, acc[ft][2 * k + 1]);
                }
            }
        }
        for (int ft = 0; ft < kFT; ++ft)
            for (int k = 0; k < 8; ++k) {
                const long long s = wave_sum64(fix32(acc[ft][k]));
                if (lane == 0) red[wv][ft * 8 + k] = s;
            }
        __syncthreads();
        if (tid < kFT * 8) {
            const int ft = tid / 8, k = tid % 8;
            if (f0 + ft < nf) {
                long long s = 0;
                for (int x = 0; x < kPoThreads / 64; ++x) s += red[x][tid];
                out[(f0 + ft) * 8 + k] = s;
            }
        }
        __syncthreads();
    }
}

// One wave per (angle, frequency): lane t sums the angle's block partials
// t, t + 64, ... in float64, the lanes are combined by a fixed xor-shuffle
// tree (the same order on every run), then A = -(k dA / 2 pi) 2^-32 S and
// sigma in dBsm.
__global__ __launch_bounds__(64) void k_po_final(PoP p, int max_nf, double *__restrict__ A_out,
                                                 double *__restrict__ sigma)
{
    const int a = static_cast<int>(blockIdx.x / max_nf), f = static_cast<int>(blockIdx.x % max_nf);
    const PoAngle &A = p.ang[a];
    if (f >= A.n_f) return;
    const int lane = threadIdx.x;
    const int64_t nch = po_units(A.rec_cnt);
    double S[8];
    for (int e = 0; e < 8; ++e) S[e] = 0.0;
    for (int64_t c = lane; c < nch; c += 64) {
        const long long *q = p.partial + (A.part_base + c * A.n_f + f) * 8;
        for (int e = 0; e < 8; ++e) S[e] += static_cast<double>(q[e]);
    }
    for (int off = 32; off >= 1; off >>= 1)
        for (int e = 0; e < 8; ++e) S[e] += __shfl_xor(S[e], off, 64);
    if (lane != 0) return;
    const double C = -(p.kf[A.kf_off + f] * A.dA / (2.0 * kPi)) * 2.3283064365386963e-10;  // 2^-32
    const int64_t row = A.out_base + f;
    double *Ao = A_out + row * 8;
    for (int k = 0; k < 4; ++k) {
        const double re = C * S[2 * k], im = C * S[2 * k + 1];
        Ao[2 * k] = re;
        Ao[2 * k + 1] = im;
        if (sigma) {
            const double sg = 4.0 * kPi * (re * re + im * im);
            sigma[row * 4 + k] = sg > 0.0 ? 10.0 * log10(sg) : -400.0;
        }
    }
}

// Caller hit e -> record slot e.
__global__ void k_pack(sbr_hits h, int64_t n, Records rec)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int fl = h.flags[e];
    if (!(fl & SBR_REC_VALID)) {
        rec.r2[e] = make_float4(0.f, 0.f, 0.f, __int_as_float(0));
        return;
    }
    rec.r0[e] = make_float4(h.d_last[3 * e], h.d_last[3 * e + 1], h.d_last[3 * e + 2], __int_as_float(h.tri_last[e]));
    rec.r1[e] = make_float4(h.eH_last[3 * e], h.eH_last[3 * e + 1], h.eH_last[3 * e + 2],
                            __int_as_float(h.tri_first[e]));
    rec.r2[e] = make_float4(h.eV_last[3 * e], h.eV_last[3 * e + 1], h.eV_last[3 * e + 2],
                            __int_as_float((h.n_bounce[e] & 255) | (fl << 8)));
    rec.D[e] = h.D[e];
}

}  // namespace

static PoP make_pop(const PoArgs &a)
{
    PoP p;
    p.rec = a.rec;
    p.ang = a.ang;
    p.n_angles = a.n_angles;
    p.nrm_id = a.bvh->nrm_id;
    p.mode = a.mode;
    p.kf = a.kf;
    p.partial = a.partial;
    return p;
}

int launch_po(hipStream_t s, const PoArgs &a)
{
    if (a.n_units <= 0) return SBR_OK;
    if (a.n_units > 2147483647LL) return fail(SBR_ERR_OVERFLOW, "PO launch: too many blocks");
    // one frequency: the 1-wide pass keeps the register count (and the
    // occupancy that hides the record loads) of a single accumulator set
    if (a.max_nf == 1) k_po<1><<<static_cast<unsigned>(a.n_units), kPoThreads, 0, s>>>(make_pop(a));
    else k_po<4><<<static_cast<unsigned>(a.n_units), kPoThreads, 0, s>>>(make_pop(a));
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_po_finalize(hipStream_t s, const PoArgs &a, double *A_out, double *sigma_out)
{
    const int64_t n = static_cast<int64_t>(a.n_angles) * a.max_nf;
    if (n > 2147483647LL) return fail(SBR_ERR_OVERFLOW, "PO finalize: too many outputs");
    k_po_final<<<static_cast<unsigned>(n), 64, 0, s>>>(make_pop(a), a.max_nf, A_out, sigma_out);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_pack_hits(hipStream_t s, const sbr_hits *h, int64_t n, Records rec)
{
    k_pack<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(*h, n, rec);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

}  // namespace sbr
