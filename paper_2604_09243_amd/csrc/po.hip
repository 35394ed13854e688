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
    const float4 *nrm_slot;
    int rec_slots;  // records name their last triangle by leaf slot (sweeps, batches) or by id (caller hits)
    int mode;
    const double *kf;
    long long *partial;
    int fp32;  // precision study: phase = fl32(fl32(k) fl32(D)), one sine and cosine per frequency
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
    // quadrant qi: (sin, cos) = (sn, cs), (cs, -sn), (-sn, -cs), (-cs, sn)
    const bool odd = qi & 1;
    const double a = odd ? cs : sn, b = odd ? sn : cs;
    so = (qi & 2) ? -a : a;
    co = ((qi + 1) & 2) ? -b : b;
}

// The precision study's single-precision phase: k and D rounded to float32,
// their product rounded to float32.
__device__ __forceinline__ double phase32(double k, double D)
{
    return static_cast<double>(static_cast<float>(k) * static_cast<float>(D));
}

// sin and cos of the phase ph (any size; float64): ph reduced by the nearest
// multiple of 2 pi (2 pi as a two-term sum), then sincos_pi.
__device__ __forceinline__ void phase_sincos(double ph, double &so, double &co)
{
    const double two_pi_hi = 6.283185307179586;       // fl64(2 pi)
    const double two_pi_lo = 2.4492935982947064e-16;  // 2 pi - fl64(2 pi)
    const double nturn = rint(ph * 0.15915494309189535);
    sincos_pi(__builtin_fma(-nturn, two_pi_lo, __builtin_fma(-nturn, two_pi_hi, ph)), so, co);
}

// (cos, sin)(m pi / 32) for m = tid < 64 into tab[m]: sincos_pi of
// j pi / 32, j = min(m mod 16, 16 - m mod 16) <= 8 (so |x| <= pi / 4), the
// rest by exact symmetries (a swap for pi / 2 - x, a quarter turn per
// m / 16).
__device__ __forceinline__ void turn_table_entry(int m, double2 *tab)
{
    const double c_hi = 0.09817477042468103;   // fl64(pi / 32)
    const double c_lo = 3.827021247335479e-18;  // pi / 32 - fl64(pi / 32)
    const int k = m >> 4, j = m & 15, jj = j <= 8 ? j : 16 - j;
    double s0, c0;
    sincos_pi(__builtin_fma(static_cast<double>(jj), c_hi, jj * c_lo), s0, c0);
    const double c = j <= 8 ? c0 : s0, s = j <= 8 ? s0 : c0;
    // times j^k (j the imaginary unit): (c, s), (-s, c), (-c, -s), (s, -c)
    tab[m] = k == 0 ? make_double2(c, s) : k == 1 ? make_double2(-s, c) : k == 2 ? make_double2(-c, -s)
                                                                              : make_double2(s, -c);
}

// sin and cos of the phase ph (float64) by the table of turn_table_entry:
// ph = q pi / 32 + r with q the nearest integer (pi / 32 as a two-term sum),
// |r| <= pi / 64, where sin r and cos r need Taylor terms up to r^9 and r^8
// (the next ones are below 1e-19); then the angle-addition formulas with
// (cos, sin)(q pi / 32) = tab[q mod 64].
__device__ __forceinline__ void phase_sincos_tab(double ph, const double2 *tab, double &so, double &co)
{
    const double c_hi = 0.09817477042468103;   // fl64(pi / 32)
    const double c_lo = 3.827021247335479e-18;  // pi / 32 - fl64(pi / 32)
    const double q = rint(ph * 10.185916357881302);  // 32 / pi
    double r = __builtin_fma(-q, c_hi, ph);
    r = __builtin_fma(-q, c_lo, r);
    const double z = r * r;
    double ps = 1.0 / 362880.0;
    ps = __builtin_fma(ps, z, -1.0 / 5040.0);
    ps = __builtin_fma(ps, z, 1.0 / 120.0);
    ps = __builtin_fma(ps, z, -1.0 / 6.0);
    const double sn = __builtin_fma(r * z, ps, r);
    double pc = 1.0 / 40320.0;
    pc = __builtin_fma(pc, z, -1.0 / 720.0);
    pc = __builtin_fma(pc, z, 1.0 / 24.0);
    pc = __builtin_fma(pc, z, -0.5);
    const double cs = __builtin_fma(z, pc, 1.0);
    const double2 t = tab[static_cast<int>(q) & 63];  // two's complement: the residue mod 64 for q < 0 too
    so = __builtin_fma(t.y, cs, t.x * sn);
    co = __builtin_fma(t.x, cs, -(t.y * sn));
}

// round(x * 2^32) as a 64-bit integer for |x| < 2^19, via the float64
// rounding of x * 2^32 + 1.5 * 2^52.
__device__ __forceinline__ long long fix32(double x)
{
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    const double y = __builtin_fma(x, 4294967296.0, magic);
    return __double_as_longlong(y) - __double_as_longlong(magic);
}

// The facet normal a record's weights use: PAPER mode the first hit's
// (r1.w: triangle id), VECTOR mode the last hit's (r0.w: leaf slot where the
// records name slots, else triangle id).
__device__ __forceinline__ float4 rec_normal(const PoP &p, const float4 r0, const float4 r1)
{
    if (p.mode == SBR_MODE_PAPER) return p.nrm_id[__float_as_int(r1.w)];
    return p.rec_slots ? p.nrm_slot[__float_as_int(r0.w)] : p.nrm_id[__float_as_int(r0.w)];
}

// Per-record weights w[p * 2 + q] in float64 from the float32 record fields:
// the cross-polar weights of VECTOR mode are differences of nearly equal
// products, and their float32 rounding, identical for the many rays of a flat
// facet, would add up coherently.  n is the record's facet normal
// (rec_normal).
__device__ __forceinline__ void weights(const PoP &p, const double *B, const float4 r0, const float4 r1,
                                        const float4 r2, const float4 n, double w[4])
{
    const int meta = __float_as_int(r2.w);
    const int N = meta & 255;
    const int flags = meta >> 8;
    w[0] = w[1] = w[2] = w[3] = 0.0;
    if (!(flags & SBR_REC_VALID)) return;
    if (p.mode == SBR_MODE_PAPER) {
        const float4 n0 = n;
        const double c0 = fabs((static_cast<double>(n0.x) * B[0] + static_cast<double>(n0.y) * B[1]) +
                               static_cast<double>(n0.z) * B[2]);
        const double s = (N & 1) ? c0 : -c0;
        w[0] = s;
        w[3] = s;
        return;
    }
    const float4 n32 = n;
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

// Angle of block u of a launch: the last angle whose first block is <= u.
__device__ __forceinline__ int po_angle_of(const PoP &p, int64_t u)
{
    int lo = 0, hi = p.n_angles;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (p.ang[mid].unit_base <= u) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Frequencies [f_begin, f_end) of records [c * kPoRecsPerBlock, (c + 1) *
// kPoRecsPerBlock) of angle A, kFT frequencies per pass over the records, in
// a block of kNT threads of which the first 256 take records: each sums the
// slots tid, tid + 256, ... (a fixed subset, in a fixed order) in float64;
// the per-thread sums become fixed point before the exact integer reduction
// over threads, waves and blocks.
template <int kFT, int kNT>
__device__ __forceinline__ void po_passes(const PoP &p, const PoAngle &A, int64_t c, int f_begin, int f_end,
                                          long long (*red)[kFT * 8])
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nf = A.n_f;
    const double *kf = p.kf + A.kf_off;
    long long *out = p.partial + (A.part_base + c * nf) * 8;
    const int64_t r0i = c * kPoRecsPerBlock;
    const int64_t r1i = tid < kPoThreads ? min(r0i + kPoRecsPerBlock, A.rec_cnt) : r0i;
    const bool f32 = p.fp32 != 0;
    const bool uniform = A.dk != 0.0 && !f32;
    for (int f0 = f_begin; f0 < f_end; f0 += kFT) {
        double acc[kFT][8];
        for (int ft = 0; ft < kFT; ++ft)
            for (int e = 0; e < 8; ++e) acc[ft][e] = 0.0;
        for (int64_t e = A.rec_base + r0i + tid; e < A.rec_base + r1i; e += kPoThreads) {
            if (!p.rec.held[e]) continue;  // no record in this slot
            const Rec &rec = p.rec.rec[e];
            const float4 q2 = rec.r2, q0 = rec.r0, q1 = rec.r1;
            const double D = rec.D.x;
            if (!((__float_as_int(q2.w) >> 8) & SBR_REC_VALID)) continue;  // dropped as trapped: no term
            double w[4];
            weights(p, A.basis, q0, q1, q2, rec_normal(p, q0, q1), w);
            double sd, cd, rs = 0.0, rc = 1.0;
            phase_sincos(f32 ? phase32(kf[f0], D) : kf[f0] * D, sd, cd);
            if (uniform) phase_sincos(A.dk * D, rs, rc);  // evenly spaced: each step turns the phasor by dk D
#pragma unroll
            for (int ft = 0; ft < kFT; ++ft) {
                const int f = f0 + ft;
                if (f >= f_end) break;
                if (ft > 0) {
                    if (uniform) {
                        const double s2 = __builtin_fma(sd, rc, cd * rs);
                        cd = __builtin_fma(cd, rc, -(sd * rs));
                        sd = s2;
                    } else {
                        phase_sincos(f32 ? phase32(kf[f], D) : kf[f] * D, sd, cd);
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
            if (f0 + ft < f_end) {
                long long s = 0;
                for (int x = 0; x < kNT / 64; ++x) s += red[x][tid];
                out[(f0 + ft) * 8 + k] = s;
            }
        }
        __syncthreads();
    }
}

// Block u of the launch: records [c * kPoRecsPerBlock, (c + 1) * kPoRecsPerBlock)
// of angle a, where a is the angle whose blocks hold u and c = u - unit_base;
// all frequencies of the angle, kFT per pass over the records.
template <int kFT>  // frequencies per pass over a block's records
__global__ __launch_bounds__(kPoThreads) void k_po(PoP p)
{
    __shared__ long long red[kPoThreads / 64][kFT * 8];
    const int64_t u = blockIdx.x;
    const PoAngle &A = p.ang[po_angle_of(p, u)];
    po_passes<kFT, kPoThreads>(p, A, u - A.unit_base, 0, A.n_f, red);
}

// Many frequencies, two kernels: k_po_mf<false> takes the angles whose
// wavenumbers are evenly spaced (step dk), k_po_mf<true> the others; each
// passes over the other's blocks at once, and the host launches only the
// kinds a call has.  Block (u, y) takes the records of unit u (as k_po) and
// the chunk of CH frequencies [CH y, CH y + CH) of its angle: evenly
// spaced 64 (8 groups of F = 8 per thread), uneven 32 (16 groups of 2).
// The rounds stage 512 record slots at a time in LDS (every field of a
// thread's two slots in one round trip, then their facet normals), the
// valid records packed in a fixed order (thread-major, then the thread's
// slots in order), with what every frequency needs computed once per
// record: the weights, D and, evenly spaced, the phasor exp(j k_fc D) at
// the chunk's first frequency and the steps exp(j s dk D) for s = 1, F,
// 2F, 4F (by repeated squaring).  So the records leave HBM once per chunk,
// not once per pass.  Uneven, the block first lists the slots that hold a
// record (one round trip over the slots' bytes) and the rounds take only
// those, so the empty slots of masked or missed rays cost no round.
// Thread t takes frequency group g = t mod G (G a power of two, as many as
// the chunk needs) and the packed records t / G, t / G + 256 / G, ... of
// every round.  Evenly spaced, a group is F consecutive frequencies: its
// phasor starts at exp(j k_fc D) turned by F g dk D (three complex
// products by a staged step or by 1) and turns by dk D per frequency.
// Uneven, the chunk is split evenly over the groups (ceil(n / G) each) and
// every frequency takes one sine and cosine (phase_sincos_tab).  A chunk of
// one frequency takes the k_po<1> summation, so single-frequency angles
// give the same bits in either kernel.
#ifndef SBR_PO_FT
#define SBR_PO_FT 8  // frequencies per thread in k_po_mf
#endif
#ifndef SBR_PO_QUNROLL
#define SBR_PO_QUNROLL 1  // packed records per iteration of the common-case loop
#endif
#ifndef SBR_PO_SUB
#define SBR_PO_SUB 512  // records staged per round in k_po_mf
#endif
constexpr int kMfFT = SBR_PO_FT, kMfChunk = 8 * kMfFT, kMfSub = SBR_PO_SUB;
constexpr int kMfLogFT = kMfFT == 2 ? 1 : kMfFT == 4 ? 2 : kMfFT == 8 ? 3 : 4;
static_assert((1 << kMfLogFT) == kMfFT, "k_po_mf: frequencies per thread must be 2, 4, 8 or 16");

__device__ __forceinline__ long long shfl_xor64(long long x, int off)
{
    const int lo = __shfl_xor(static_cast<int>(x), off, 64);
    const int hi = __shfl_xor(static_cast<int>(x >> 32), off, 64);
    return static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                  static_cast<unsigned>(lo));
}

// Frequencies per thread, blocks per CU and frequency groups per block of
// the uneven-spacing kernel: there every frequency takes its own sine and
// cosine, so a record's LDS reads are a small part of its work per
// frequency, and 2 frequencies per thread (a quarter of the accumulators of
// 8) buy four blocks per CU, with up to 16 groups so that a chunk is still
// 32 frequencies (its records staged once).
#ifndef SBR_PO_FTU
#define SBR_PO_FTU 2  // frequencies per thread, uneven spacing
#endif
#ifndef SBR_PO_BLOCKSU
#define SBR_PO_BLOCKSU 4  // blocks per CU, uneven spacing
#endif
#ifndef SBR_PO_GROUPSU
#define SBR_PO_GROUPSU 16  // at most this many frequency groups per block, uneven spacing
#endif
constexpr int kMfFTu = SBR_PO_FTU, kMfBlocksU = SBR_PO_BLOCKSU, kMfGroupsU = SBR_PO_GROUPSU;

template <bool kUneven>  // the angles of the launch it takes: evenly spaced (false) or not (true)
__global__ __launch_bounds__(kPoThreads, kUneven ? kMfBlocksU : 2) void k_po_mf(PoP p)
{
    constexpr int FT = kUneven ? kMfFTu : kMfFT;  // frequencies per thread
    constexpr int GM = kUneven ? kMfGroupsU : 8;  // frequency groups per block, at most
    constexpr int CH = GM * FT;                   // frequencies per block
    __shared__ double sw[4][kMfSub];              // weights
    __shared__ double sD[kMfSub];                 // path length
    // evenly spaced: (cos, sin) of k_fc D, dk D, F dk D, 2F dk D, 4F dk D (F = kMfFT)
    __shared__ double sph[kUneven ? 1 : 10][kUneven ? 1 : kMfSub];
    __shared__ double skf[CH];                    // uneven: the chunk's wavenumbers
    __shared__ double2 stab[kUneven ? 64 : 1];    // uneven: (cos, sin)(m pi / 32)
    __shared__ int scnt[kPoThreads / 64];
    __shared__ long long red[kPoThreads / 64][CH * 8];
    const int64_t u = blockIdx.x;
    const PoAngle &A = p.ang[po_angle_of(p, u)];
    const bool uniform = A.dk != 0.0;
    if (uniform == kUneven) return;  // the other kernel's angle
    const int nf = A.n_f;
    const int fc = static_cast<int>(blockIdx.y) * CH;
    if (fc >= nf) return;  // the whole block
    const int nfc = min(CH, nf - fc);
    const int64_t c = u - A.unit_base;
    if (nfc == 1) {
        po_passes<1, kPoThreads>(p, A, c, fc, fc + 1, reinterpret_cast<long long (*)[8]>(&red[0][0]));
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int lg = 0;  // G = 2^lg groups of FT cover the chunk (lg <= 3 evenly spaced: the staged steps)
    while ((FT << lg) < nfc) ++lg;
    const int G = 1 << lg, g = tid & (G - 1), rl = tid >> lg, RL = kPoThreads >> lg;
    // frequencies per group: evenly spaced F (the staged steps F, 2F, 4F
    // start the groups' phasors) unless one group takes the chunk, uneven
    // the chunk split evenly over the groups
    const int nfg = !kUneven && lg > 0 ? FT : (nfc + G - 1) >> lg;
    const int fs = fc + g * nfg;                       // this thread's first frequency
    const int nft = max(0, min(nfg, fc + nfc - fs));  // and how many
    const double *kf = p.kf + A.kf_off;
    const int64_t r0i = c * kPoRecsPerBlock;
    const int64_t r1i = min(r0i + kPoRecsPerBlock, A.rec_cnt);
    if constexpr (kUneven) {  // 0 past the chunk's end: summed by the idle slots of the last group, never stored
        for (int i = tid; i < CH; i += kPoThreads) skf[i] = i < nfc ? kf[fc + i] : 0.0;
        if (tid < 64) turn_table_entry(tid, stab);
    }
    double acc[FT][8];
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[ft][e] = 0.0;
    // Uneven spacing: the block's slots that hold a record, listed once
    // (their bytes in one round trip: slot r0i + i 256 + t read by thread
    // t), in a fixed order (thread-major, then i); the rounds below then
    // stage only those, so the empty slots of masked or missed rays cost
    // neither rounds nor round trips.  The list lives in the reduction
    // buffer, unused until the last round has ended.  Evenly spaced, the
    // rounds take the slots as they come: a list costs those blocks more
    // registers than the rounds it saves (their records fill most slots).
    uint16_t *slist = reinterpret_cast<uint16_t *>(&red[0][0]);
    static_assert(!kUneven || sizeof(red) >= kPoRecsPerBlock * sizeof(uint16_t), "k_po_mf: slot list does not fit");
    static_assert(kPoRecsPerBlock <= 65536, "k_po_mf: slot offsets are 16-bit");
    int nheld = static_cast<int>(r1i - r0i);
    long long *out = p.partial + (A.part_base + c * nf + fc) * 8;
    if constexpr (kUneven) {
        nheld = 0;
        constexpr int kSpt = kPoRecsPerBlock / kPoThreads;
        static_assert(kSpt <= 32, "k_po_mf: a thread's slots are one 32-bit mask");
        uint32_t hm = 0;
#pragma unroll
        for (int i = 0; i < kSpt; ++i) {
            const int64_t e = r0i + i * kPoThreads + tid;
            if (e < r1i && p.rec.held[A.rec_base + e] != 0) hm |= 1u << i;
        }
        const int hc = __popc(hm);
        int inc = hc;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(inc, off, 64);
            if (lane >= off) inc += v;
        }
        if (lane == 63) scnt[wv] = inc;
        __syncthreads();
        int pos = inc - hc;
        for (int x = 0; x < kPoThreads / 64; ++x) {
            if (x < wv) pos += scnt[x];
            nheld += scnt[x];
        }
        for (int i = 0; hm != 0; ++i, hm >>= 1)
            if (hm & 1) slist[pos++] = static_cast<uint16_t>(i * kPoThreads + tid);
        __syncthreads();
        if (nheld == 0) {  // no record (the same for every thread): zero sums without the reduction
            for (int i = tid; i < nfc * 8; i += kPoThreads) out[i] = 0;
            return;
        }
    }
    for (int s0 = 0; s0 < nheld; s0 += kMfSub) {
        // stage: thread t holds list entries (uneven) or slots (evenly
        // spaced) s0 + t + 256 j, j = 0, 1
        constexpr int kPer = kMfSub / kPoThreads;
        int vmask = 0, cnt = 0;
        // every field of the listed slots at once (one round trip), then the
        // facet normals the weights need
        float4 q0[kPer], q1[kPer], q2[kPer];
        double Dj[kPer];
        bool held[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int x = s0 + tid + j * kPoThreads;
            held[j] = x < nheld && (kUneven || p.rec.held[A.rec_base + r0i + x] != 0);
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (held[j]) {
                const int x = s0 + tid + j * kPoThreads;
                const int64_t ea = A.rec_base + r0i + (kUneven ? slist[x] : x);
                const Rec &rec = p.rec.rec[ea];
                q0[j] = rec.r0;
                q1[j] = rec.r1;
                q2[j] = rec.r2;
                Dj[j] = rec.D.x;
            }
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (held[j] && ((__float_as_int(q2[j].w) >> 8) & SBR_REC_VALID)) {
                vmask |= 1 << j;
                ++cnt;
            }
        }
        // exclusive scan of the counts over the block (thread order)
        int inc = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(inc, off, 64);
            if (lane >= off) inc += v;
        }
        if (lane == 63) scnt[wv] = inc;
        __syncthreads();
        int pos = inc - cnt, nvalid = 0;
        for (int x = 0; x < kPoThreads / 64; ++x) {
            if (x < wv) pos += scnt[x];
            nvalid += scnt[x];
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (!((vmask >> j) & 1)) continue;
            const double D = Dj[j];
            double w[4];
            weights(p, A.basis, q0[j], q1[j], q2[j], rec_normal(p, q0[j], q1[j]), w);
            for (int k = 0; k < 4; ++k) sw[k][pos] = w[k];
            sD[pos] = D;
            if constexpr (!kUneven) {
                double bs, bc, rs, rc;
                phase_sincos(kf[fc] * D, bs, bc);
                phase_sincos(A.dk * D, rs, rc);
                sph[0][pos] = bc;
                sph[1][pos] = bs;
                sph[2][pos] = rc;
                sph[3][pos] = rs;
                // (rc + j rs)^F, ^2F, ^4F (F = kMfFT) by repeated squaring
                for (int sq = 1; sq <= kMfLogFT + 2; ++sq) {
                    const double c2 = __builtin_fma(rc, rc, -(rs * rs)), s2 = 2.0 * (rc * rs);
                    rc = c2;
                    rs = s2;
                    if (sq >= kMfLogFT) {
                        sph[4 + 2 * (sq - kMfLogFT)][pos] = rc;
                        sph[5 + 2 * (sq - kMfLogFT)][pos] = rs;
                    }
                }
            }
            ++pos;
        }
        __syncthreads();
        if constexpr (kUneven) {
            // one sine and cosine per frequency; every thread takes nfg
            // (a trip count the same for the whole block)
            const double *kq = skf + (fs - fc);
            for (int q = rl; q < nvalid; q += RL) {
                const double w0 = sw[0][q], w1 = sw[1][q], w2 = sw[2][q], w3 = sw[3][q];
                const double D = sD[q];
#pragma unroll
                for (int ft = 0; ft < FT; ++ft) {
                    if (ft >= nfg) break;
                    double sd, cd;
                    phase_sincos_tab(kq[ft] * D, stab, sd, cd);
                    acc[ft][0] = __builtin_fma(w0, sd, acc[ft][0]);
                    acc[ft][1] = __builtin_fma(w0, cd, acc[ft][1]);
                    acc[ft][2] = __builtin_fma(w1, sd, acc[ft][2]);
                    acc[ft][3] = __builtin_fma(w1, cd, acc[ft][3]);
                    acc[ft][4] = __builtin_fma(w2, sd, acc[ft][4]);
                    acc[ft][5] = __builtin_fma(w2, cd, acc[ft][5]);
                    acc[ft][6] = __builtin_fma(w3, sd, acc[ft][6]);
                    acc[ft][7] = __builtin_fma(w3, cd, acc[ft][7]);
                }
            }
        } else if (nft == FT) {
            // the common case, branch free: a full group
#pragma unroll SBR_PO_QUNROLL
            for (int q = rl; q < nvalid; q += RL) {
                const double w0 = sw[0][q], w1 = sw[1][q], w2 = sw[2][q], w3 = sw[3][q];
                double cd = sph[0][q], sd = sph[1][q];
                const double rc = sph[2][q], rs = sph[3][q];
                // start at frequency fc + F g: turn by F g dk D (g < 8: the staged steps F, 2F, 4F;
                // bits of g at or above lg are 0, a turn by exactly 1)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    if (b >= lg) break;
                    // by the step (tc, ts) or by 1 (exactly: 0 t + 1 and 0 t), without a branch
                    const double on = static_cast<double>((g >> b) & 1);
                    const double tc = __builtin_fma(on, sph[4 + 2 * b][q], 1.0 - on), ts = on * sph[5 + 2 * b][q];
                    const double c2 = __builtin_fma(cd, tc, -(sd * ts));
                    sd = __builtin_fma(cd, ts, sd * tc);
                    cd = c2;
                }
#pragma unroll
                for (int ft = 0; ft < FT; ++ft) {
                    if (ft > 0) {
                        const double s2 = __builtin_fma(sd, rc, cd * rs);
                        cd = __builtin_fma(cd, rc, -(sd * rs));
                        sd = s2;
                    }
                    acc[ft][0] = __builtin_fma(w0, sd, acc[ft][0]);
                    acc[ft][1] = __builtin_fma(w0, cd, acc[ft][1]);
                    acc[ft][2] = __builtin_fma(w1, sd, acc[ft][2]);
                    acc[ft][3] = __builtin_fma(w1, cd, acc[ft][3]);
                    acc[ft][4] = __builtin_fma(w2, sd, acc[ft][4]);
                    acc[ft][5] = __builtin_fma(w2, cd, acc[ft][5]);
                    acc[ft][6] = __builtin_fma(w3, sd, acc[ft][6]);
                    acc[ft][7] = __builtin_fma(w3, cd, acc[ft][7]);
                }
            }
        } else if (nft > 0) {
            // a group of fewer than F frequencies
            for (int q = rl; q < nvalid; q += RL) {
                const double w0 = sw[0][q], w1 = sw[1][q], w2 = sw[2][q], w3 = sw[3][q];
                double cd = sph[0][q], sd = sph[1][q];
                const double rc = sph[2][q], rs = sph[3][q];
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    if (b >= lg) break;
                    const bool on = (g >> b) & 1;
                    const double tc = on ? sph[4 + 2 * b][q] : 1.0, ts = on ? sph[5 + 2 * b][q] : 0.0;
                    const double c2 = __builtin_fma(cd, tc, -(sd * ts));
                    sd = __builtin_fma(cd, ts, sd * tc);
                    cd = c2;
                }
#pragma unroll
                for (int ft = 0; ft < FT; ++ft) {
                    if (ft >= nft) break;
                    if (ft > 0) {
                        const double s2 = __builtin_fma(sd, rc, cd * rs);
                        cd = __builtin_fma(cd, rc, -(sd * rs));
                        sd = s2;
                    }
                    acc[ft][0] = __builtin_fma(w0, sd, acc[ft][0]);
                    acc[ft][1] = __builtin_fma(w0, cd, acc[ft][1]);
                    acc[ft][2] = __builtin_fma(w1, sd, acc[ft][2]);
                    acc[ft][3] = __builtin_fma(w1, cd, acc[ft][3]);
                    acc[ft][4] = __builtin_fma(w2, sd, acc[ft][4]);
                    acc[ft][5] = __builtin_fma(w2, cd, acc[ft][5]);
                    acc[ft][6] = __builtin_fma(w3, sd, acc[ft][6]);
                    acc[ft][7] = __builtin_fma(w3, cd, acc[ft][7]);
                }
            }
        }
        __syncthreads();  // before the next round overwrites the stage
    }
    // fixed point, summed over the lanes of a group (lane = g mod G) of each
    // wave, then over the waves; group g's sums at red[(g FT + ft) 8 + k]
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            long long v = fix32(acc[ft][k]);
            for (int off = 32; off >= G; off >>= 1) v += shfl_xor64(v, off);
            if (lane < G) red[wv][(lane * FT + ft) * 8 + k] = v;
        }
    __syncthreads();
    for (int i = tid; i < nfc * 8; i += kPoThreads) {
        int at = i;  // evenly spaced: nfg = F, or one group
        if constexpr (kUneven) {
            const int f = i >> 3, gf = f / nfg;  // frequency fc + f: group gf, its (f - gf nfg)-th
            at = ((gf * FT + f - gf * nfg) << 3) | (i & 7);
        }
        long long v = 0;
        for (int x = 0; x < kPoThreads / 64; ++x) v += red[x][at];
        out[i] = v;
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

// Caller hit e -> record slot e (its byte says whether it holds a record).
__global__ void k_pack(sbr_hits h, int64_t n, Records rec)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int fl = h.flags[e];
    const bool valid = (fl & SBR_REC_VALID) != 0;
    rec.held[e] = valid ? 1 : 0;
    if (!valid) return;
    Rec &q = rec.rec[e];
    q.r0 = make_float4(h.d_last[3 * e], h.d_last[3 * e + 1], h.d_last[3 * e + 2], __int_as_float(h.tri_last[e]));
    q.r1 = make_float4(h.eH_last[3 * e], h.eH_last[3 * e + 1], h.eH_last[3 * e + 2],
                            __int_as_float(h.tri_first[e]));
    q.r2 = make_float4(h.eV_last[3 * e], h.eV_last[3 * e + 1], h.eV_last[3 * e + 2],
                            __int_as_float((h.n_bounce[e] & 255) | (fl << 8)));
    q.D = make_double2(h.D[e], 0.0);
}

}  // namespace

static PoP make_pop(const PoArgs &a)
{
    PoP p;
    p.rec = a.rec;
    p.ang = a.ang;
    p.n_angles = a.n_angles;
    p.nrm_id = a.bvh->nrm_id;
    p.nrm_slot = a.bvh->nrm_slot;
    p.rec_slots = a.rec_slots;
    p.mode = a.mode;
    p.kf = a.kf;
    p.partial = a.partial;
    p.fp32 = a.fp32;
    return p;
}

int launch_po(hipStream_t s, const PoArgs &a)
{
    if (a.n_units <= 0) return SBR_OK;
    if (a.n_units > 2147483647LL) return fail(SBR_ERR_OVERFLOW, "PO launch: too many blocks");
    // one frequency: the 1-wide pass keeps the register count (and the
    // occupancy that hides the record loads) of a single accumulator set
    if (a.max_nf == 1 || a.fp32) {  // the precision study takes every frequency's phase on its own
        k_po<1><<<static_cast<unsigned>(a.n_units), kPoThreads, 0, s>>>(make_pop(a));
    } else {
        // each kernel passes over the other kind's blocks at once
        if (a.kinds != kPoUneven) {
            const dim3 grid(static_cast<unsigned>(a.n_units), static_cast<unsigned>((a.max_nf + kMfChunk - 1) / kMfChunk));
            k_po_mf<false><<<grid, kPoThreads, 0, s>>>(make_pop(a));
        }
        if (a.kinds != kPoEven) {
            constexpr int ch = kMfGroupsU * kMfFTu;
            const dim3 grid(static_cast<unsigned>(a.n_units), static_cast<unsigned>((a.max_nf + ch - 1) / ch));
            k_po_mf<true><<<grid, kPoThreads, 0, s>>>(make_pop(a));
        }
    }
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
