// Multi-bounce ray transport (Algorithm 2) on gfx950.
//
// Wavefront organisation: one kernel launch per bounce.  Bounce 1 takes its
// rays either from the incidence-angle plans (the orthographic grid of
// Eqs. L1-L3, generated in-register, 8x8 aperture tiles per 64-lane wave) or
// from caller arrays; later bounces take them from a queue.  Rays that hit
// and have bounces left are appended to the next queue with one atomic per
// wave (ballot + prefix popcount); every hit overwrites the ray's hit record,
// so the record of a terminated ray is its last hit.
//
// Launches are persistent: a fixed grid of waves pulls 64-ray tiles from
// eight counters, one per XCD-sized range of tiles (a block's XCD is taken as
// blockIdx % 8, the order in which workgroups are spread over the dies), and
// steals from the other ranges once its own is empty.
//
// Closest hit: BVH2 traversal, both child boxes of a node per 64-byte fetch,
// nearer child first, the farther one on a per-lane stack that lives in LDS
// (spilling to a global array beyond kStackLds entries).  The triangle test
// and the reflection arithmetic follow the float32 specification shared with
// the CPU oracle; this file is compiled with -ffp-contract=off, and fused
// multiply-adds are written explicitly only in the (conservative) box test.
#include <cmath>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

constexpr int kBlock = 256;
constexpr int kStackLds = 24;
constexpr int kTileRays = 64;

// stat slots
enum { ST_QUERIES = 0, ST_TRAPPED = 1, ST_VALID = 2, ST_HITS = 8 };

struct Params {
    const BNode *nodes;
    const BTri *tris;
    const float4 *nrm;  // by slot
    float eps, slack;
    int bmax;
    uint32_t flags;
    // grid source
    const AnglePlan *plans;
    const int64_t *tile_base;
    int n_angles;
    // user source / sink
    const float *uo, *ud, *uh, *uv;
    int64_t n_rays;
    sbr_hits hits;
    double kx, ky, kz;
    // queues
    RayQueue qin, qout;
    const uint32_t *qin_cnt;
    uint32_t *qout_cnt;
    // records (compact sink)
    Records rec;
    uint32_t *rec_cnt;
    // misc
    int64_t n_tiles;  // for grid/user sources
    uint32_t *ctr;    // 8 tile counters for this launch
    unsigned long long *stat;
    int32_t *spill;
    int bounce;
    int user_sink;
};

struct Ray {
    float ox, oy, oz, dx, dy, dz;
    float hx, hy, hz, vx, vy, vz;
    int prev, first, id, meta;
    double P, comp, kdo;
    int rec;
};

__device__ __forceinline__ bool tri_test(const BTri &tr, const Ray &r, float &t_out)
{
    const float e1x = tr.p1.x, e1y = tr.p1.y, e1z = tr.p1.z;
    const float e2x = tr.p2.x, e2y = tr.p2.y, e2z = tr.p2.z;
    const float px = r.dy * e2z - r.dz * e2y;
    const float py = r.dz * e2x - r.dx * e2z;
    const float pz = r.dx * e2y - r.dy * e2x;
    const float det = (e1x * px + e1y * py) + e1z * pz;
    if (det == 0.0f) return false;
    const float sx = r.ox - tr.p0.x, sy = r.oy - tr.p0.y, sz = r.oz - tr.p0.z;
    const float un = (sx * px + sy * py) + sz * pz;
    const float qx = sy * e1z - sz * e1y;
    const float qy = sz * e1x - sx * e1z;
    const float qz = sx * e1y - sy * e1x;
    const float vn = (r.dx * qx + r.dy * qy) + r.dz * qz;
    const float tn = (e2x * qx + e2y * qy) + e2z * qz;
    const float inv = 1.0f / det;
    const float u = un * inv, v = vn * inv, t = tn * inv;
    t_out = t;
    return u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t > 0.0f && t < INFINITY;
}

struct Best {
    float t;
    int id;
    int slot;
};

__device__ __forceinline__ void leaf(const Params &p, int slot, const Ray &r, Best &b)
{
    const BTri tr = p.tris[slot];
    const int id = __float_as_int(tr.p0.w);
    if (id == r.prev) return;
    float t;
    if (tri_test(tr, r, t) && (t < b.t || (t == b.t && id < b.id))) {
        b.t = t;
        b.id = id;
        b.slot = slot;
    }
}

// Closest hit of ray r, skipping triangle r.prev.  lst: this lane's LDS stack
// column (stride kBlock); gst: its spill column (stride gstride).
__device__ Best closest(const Params &p, const Ray &r, int *lst, int32_t *gst, int64_t gstride)
{
    Best b;
    b.t = INFINITY;
    b.id = 0x7fffffff;
    b.slot = -1;
    const float tiny = 1e-20f;
    const float ddx = fabsf(r.dx) < tiny ? copysignf(tiny, r.dx) : r.dx;
    const float ddy = fabsf(r.dy) < tiny ? copysignf(tiny, r.dy) : r.dy;
    const float ddz = fabsf(r.dz) < tiny ? copysignf(tiny, r.dz) : r.dz;
    const float ix = __builtin_amdgcn_rcpf(ddx), iy = __builtin_amdgcn_rcpf(ddy), iz = __builtin_amdgcn_rcpf(ddz);
    const float ox = r.ox * ix, oy = r.oy * iy, oz = r.oz * iz;
    int sp = 0;
    int node = 0;
    for (;;) {
        const BNode n = p.nodes[node];
        const float tlim = __builtin_fmaf(b.t, 1.000001f, p.slack);
        // child 0: lo = (a.x, a.y, a.z), hi = (a.w, b.x, b.y)
        const float ax0 = __builtin_fmaf(n.a.x, ix, -ox), ax1 = __builtin_fmaf(n.a.w, ix, -ox);
        const float ay0 = __builtin_fmaf(n.a.y, iy, -oy), ay1 = __builtin_fmaf(n.b.x, iy, -oy);
        const float az0 = __builtin_fmaf(n.a.z, iz, -oz), az1 = __builtin_fmaf(n.b.y, iz, -oz);
        const float t0 = fmaxf(fmaxf(fminf(ax0, ax1), fminf(ay0, ay1)), fmaxf(fminf(az0, az1), 0.0f));
        const float u0 = fminf(fminf(fmaxf(ax0, ax1), fmaxf(ay0, ay1)), fminf(fmaxf(az0, az1), tlim));
        // child 1: lo = (b.z, b.w, c.x), hi = (c.y, c.z, c.w)
        const float bx0 = __builtin_fmaf(n.b.z, ix, -ox), bx1 = __builtin_fmaf(n.c.y, ix, -ox);
        const float by0 = __builtin_fmaf(n.b.w, iy, -oy), by1 = __builtin_fmaf(n.c.z, iy, -oy);
        const float bz0 = __builtin_fmaf(n.c.x, iz, -oz), bz1 = __builtin_fmaf(n.c.w, iz, -oz);
        const float t1 = fmaxf(fmaxf(fminf(bx0, bx1), fminf(by0, by1)), fmaxf(fminf(bz0, bz1), 0.0f));
        const float u1 = fminf(fminf(fmaxf(bx0, bx1), fmaxf(by0, by1)), fminf(fmaxf(bz0, bz1), tlim));
        bool h0 = t0 <= u0, h1 = t1 <= u1;
        int c0 = n.ch.x, c1 = n.ch.y;
        if (h0 && c0 < 0) {
            leaf(p, ~c0, r, b);
            h0 = false;
        }
        if (h1 && c1 < 0) {
            leaf(p, ~c1, r, b);
            h1 = false;
        }
        if (h0 && h1) {
            int nr = c0, fr = c1;
            if (t1 < t0) {
                nr = c1;
                fr = c0;
            }
            if (sp < kStackLds) lst[sp * kBlock] = fr;
            else gst[(sp - kStackLds) * gstride] = fr;
            ++sp;
            node = nr;
        } else if (h0) {
            node = c0;
        } else if (h1) {
            node = c1;
        } else {
            if (sp == 0) break;
            --sp;
            node = sp < kStackLds ? lst[sp * kBlock] : gst[(sp - kStackLds) * gstride];
        }
    }
    return b;
}

__device__ __forceinline__ double dotk(const Params &p, const double *k, float x, float y, float z)
{
    return (k[0] * static_cast<double>(x) + k[1] * static_cast<double>(y)) + k[2] * static_cast<double>(z);
}

__device__ __forceinline__ int64_t fetch_tile(uint32_t *ctr, int64_t n_tiles, int xcd)
{
    for (int kk = 0; kk < 8; ++kk) {
        const int c = (xcd + kk) & 7;
        const int64_t lo = n_tiles * c / 8, hi = n_tiles * (c + 1) / 8;
        if (hi <= lo) continue;
        const uint32_t t = atomicAdd(&ctr[c], 1u);
        if (lo + static_cast<int64_t>(t) < hi) return lo + t;
    }
    return -1;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = threadIdx.x & 63;
    return (1ull << lane) - 1ull;
}

// Wave-aggregated atomic add: every active lane with `want` gets a distinct
// slot from *ctr (consecutive within the wave, in lane order).
__device__ __forceinline__ uint32_t wave_alloc(uint32_t *ctr, bool want, uint64_t &mask_out)
{
    const uint64_t m = __ballot(want);
    mask_out = m;
    uint32_t base = 0;
    if (m) {
        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
        if ((threadIdx.x & 63) == leader) base = atomicAdd(ctr, static_cast<uint32_t>(__popcll(m)));
        base = __shfl(base, leader);
    }
    return base + static_cast<uint32_t>(__popcll(m & lanemask_lt()));
}

template <int SRC>  // 0 = angle grid, 1 = caller rays, 2 = queue
__global__ __launch_bounds__(kBlock) void k_trace(Params p)
{
    __shared__ int lds_stack[kStackLds * kBlock];
    int *lst = lds_stack + threadIdx.x;
    const int64_t gstride = static_cast<int64_t>(gridDim.x) * kBlock;
    int32_t *gst = p.spill + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int xcd = blockIdx.x & 7;
    const bool drop_trapped = (p.flags & SBR_OPT_DROP_TRAPPED) != 0;
    const bool paper_path = (p.flags & SBR_OPT_PAPER_PATH) != 0;
    int64_t n_tiles = p.n_tiles;
    uint32_t n_in = 0;
    if (SRC == 2) {
        n_in = *p.qin_cnt;
        n_tiles = (static_cast<int64_t>(n_in) + kTileRays - 1) / kTileRays;
    }
    unsigned long long my_queries = 0, my_hits = 0, my_trapped = 0;

    for (;;) {
        int64_t tile = 0;
        if (lane == 0) tile = fetch_tile(p.ctr, n_tiles, xcd);
        tile = __shfl(tile, 0);
        if (tile < 0) break;

        Ray r;
        bool active;
        int slot = 0;
        const double *kv = nullptr;
        double kloc[3];
        if (SRC == 0) {
            int lo = 0, hi = p.n_angles;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (p.tile_base[mid] <= tile) lo = mid;
                else hi = mid;
            }
            slot = lo;
            const AnglePlan &pl = p.plans[slot];
            const int64_t t = tile - pl.tile_base;
            const int i = static_cast<int>(t % pl.tu) * 8 + (lane & 7);
            const int j = static_cast<int>(t / pl.tu) * 8 + (lane >> 3);
            active = i < pl.nu && j < pl.nv;
            const double ui = pl.uc + ((static_cast<double>(i) + 0.5) - 0.5 * static_cast<double>(pl.nu)) * pl.ds;
            const double vj = pl.vc + ((static_cast<double>(j) + 0.5) - 0.5 * static_cast<double>(pl.nv)) * pl.ds;
            r.ox = static_cast<float>((ui * pl.u[0] + vj * pl.v[0]) + pl.s0 * pl.k[0]);
            r.oy = static_cast<float>((ui * pl.u[1] + vj * pl.v[1]) + pl.s0 * pl.k[1]);
            r.oz = static_cast<float>((ui * pl.u[2] + vj * pl.v[2]) + pl.s0 * pl.k[2]);
            r.dx = pl.d32[0];
            r.dy = pl.d32[1];
            r.dz = pl.d32[2];
            r.hx = pl.eH32[0];
            r.hy = pl.eH32[1];
            r.hz = pl.eH32[2];
            r.vx = pl.eV32[0];
            r.vy = pl.eV32[1];
            r.vz = pl.eV32[2];
            r.prev = -1;
            r.first = -1;
            r.id = j * pl.nu + i;
            r.meta = slot << 8;
            r.P = 0.0;
            r.comp = 0.0;
            kv = pl.k;
            r.kdo = dotk(p, kv, r.ox, r.oy, r.oz);
            r.rec = -1;
        } else if (SRC == 1) {
            const int64_t e = tile * kTileRays + lane;
            active = e < p.n_rays;
            const int64_t ee = active ? e : 0;
            r.ox = p.uo[3 * ee];
            r.oy = p.uo[3 * ee + 1];
            r.oz = p.uo[3 * ee + 2];
            r.dx = p.ud[3 * ee];
            r.dy = p.ud[3 * ee + 1];
            r.dz = p.ud[3 * ee + 2];
            r.hx = p.uh[3 * ee];
            r.hy = p.uh[3 * ee + 1];
            r.hz = p.uh[3 * ee + 2];
            r.vx = p.uv[3 * ee];
            r.vy = p.uv[3 * ee + 1];
            r.vz = p.uv[3 * ee + 2];
            r.prev = -1;
            r.first = -1;
            r.id = static_cast<int>(ee);
            r.meta = 0;
            r.P = 0.0;
            r.comp = 0.0;
            kloc[0] = p.kx;
            kloc[1] = p.ky;
            kloc[2] = p.kz;
            kv = kloc;
            r.kdo = dotk(p, kv, r.ox, r.oy, r.oz);
            r.rec = -1;
        } else {
            const int64_t e = tile * kTileRays + lane;
            active = e < static_cast<int64_t>(n_in);
            const int64_t ee = active ? e : 0;
            const float4 s0 = p.qin.s0[ee], s1 = p.qin.s1[ee], s2 = p.qin.s2[ee], s3 = p.qin.s3[ee];
            const double2 s4 = p.qin.s4[ee], s5 = p.qin.s5[ee];
            r.ox = s0.x;
            r.oy = s0.y;
            r.oz = s0.z;
            r.prev = __float_as_int(s0.w);
            r.dx = s1.x;
            r.dy = s1.y;
            r.dz = s1.z;
            r.first = __float_as_int(s1.w);
            r.hx = s2.x;
            r.hy = s2.y;
            r.hz = s2.z;
            r.id = __float_as_int(s2.w);
            r.vx = s3.x;
            r.vy = s3.y;
            r.vz = s3.z;
            r.meta = __float_as_int(s3.w);
            r.P = s4.x;
            r.comp = s4.y;
            r.kdo = s5.x;
            r.rec = static_cast<int>(__double_as_longlong(s5.y));
            slot = r.meta >> 8;
            if (p.user_sink) {
                kloc[0] = p.kx;
                kloc[1] = p.ky;
                kloc[2] = p.kz;
                kv = kloc;
            } else {
                kv = p.plans[slot].k;
            }
        }

        // ---- closest hit
        Best b;
        b.slot = -1;
        if (active) b = closest(p, r, lst, gst, gstride);
        const bool hit = active && b.slot >= 0;
        my_queries += active ? 1 : 0;
        my_hits += hit ? 1 : 0;

        // ---- bounce update (Algorithm 2) and record of the last hit
        int N = r.meta & 127;
        bool cont = false;
        int flags = 0;
        float dlx = 0, dly = 0, dlz = 0, xlx = 0, xly = 0, xlz = 0;
        float hlx = 0, hly = 0, hlz = 0, vlx = 0, vly = 0, vlz = 0;
        double D = 0.0;
        if (hit) {
            const float t = b.t;
            xlx = r.ox + t * r.dx;
            xly = r.oy + t * r.dy;
            xlz = r.oz + t * r.dz;
            r.P = r.P + static_cast<double>(t);
            if (N >= 1 && !paper_path) r.P = r.P + r.comp;
            N += 1;
            if (N == 1) r.first = b.id;
            dlx = r.dx;
            dly = r.dy;
            dlz = r.dz;
            hlx = r.hx;
            hly = r.hy;
            hlz = r.hz;
            vlx = r.vx;
            vly = r.vy;
            vlz = r.vz;
            const float4 n = p.nrm[b.slot];
            const float dn = (r.dx * n.x + r.dy * n.y) + r.dz * n.z;
            const bool back = !(dn < 0.0f);
            const float nfx = back ? -n.x : n.x, nfy = back ? -n.y : n.y, nfz = back ? -n.z : n.z;
            const float s = 2.0f * dn;
            r.dx = r.dx - s * n.x;
            r.dy = r.dy - s * n.y;
            r.dz = r.dz - s * n.z;
            const float cH = 2.0f * ((n.x * r.hx + n.y * r.hy) + n.z * r.hz);
            const float cV = 2.0f * ((n.x * r.vx + n.y * r.vy) + n.z * r.vz);
            r.hx = cH * n.x - r.hx;
            r.hy = cH * n.y - r.hy;
            r.hz = cH * n.z - r.hz;
            r.vx = cV * n.x - r.vx;
            r.vy = cV * n.y - r.vy;
            r.vz = cV * n.z - r.vz;
            r.ox = xlx + p.eps * nfx;
            r.oy = xly + p.eps * nfy;
            r.oz = xlz + p.eps * nfz;
            r.comp = static_cast<double>(p.eps) *
                     ((static_cast<double>(nfx) * r.dx + static_cast<double>(nfy) * r.dy) +
                      static_cast<double>(nfz) * r.dz);
            r.prev = b.id;
            r.meta = (r.meta & ~0xff) | N | (back ? 128 : 0);
            D = (r.kdo + r.P) + dotk(p, kv, xlx, xly, xlz);
            flags = SBR_REC_VALID | (back ? SBR_REC_BACK_LAST : 0);
            cont = N < p.bmax;
            if (!cont && drop_trapped) {
                const Best b2 = closest(p, r, lst, gst, gstride);
                my_queries += 1;
                if (b2.slot >= 0) {
                    flags = (flags | SBR_REC_TRAPPED) & ~SBR_REC_VALID;
                    my_trapped += 1;
                }
            }
        }

        // ---- record sink
        if (p.user_sink) {
            const sbr_hits &h = p.hits;
            const int64_t e = r.id;
            if (hit) {
                if (h.n_bounce) h.n_bounce[e] = N;
                if (h.tri_first) h.tri_first[e] = r.first;
                if (h.tri_last) h.tri_last[e] = b.id;
                if (h.flags) h.flags[e] = flags;
                if (h.path) h.path[e] = r.P;
                if (h.D) h.D[e] = D;
                if (h.d_last) { h.d_last[3 * e] = dlx; h.d_last[3 * e + 1] = dly; h.d_last[3 * e + 2] = dlz; }
                if (h.x_last) { h.x_last[3 * e] = xlx; h.x_last[3 * e + 1] = xly; h.x_last[3 * e + 2] = xlz; }
                if (h.eH_last) { h.eH_last[3 * e] = hlx; h.eH_last[3 * e + 1] = hly; h.eH_last[3 * e + 2] = hlz; }
                if (h.eV_last) { h.eV_last[3 * e] = vlx; h.eV_last[3 * e + 1] = vly; h.eV_last[3 * e + 2] = vlz; }
                if (h.tri_path) h.tri_path[e * p.bmax + (N - 1)] = b.id;
            }
            if (SRC == 1 && active) {
                if (!hit) {
                    if (h.n_bounce) h.n_bounce[e] = 0;
                    if (h.tri_first) h.tri_first[e] = -1;
                    if (h.tri_last) h.tri_last[e] = -1;
                    if (h.flags) h.flags[e] = 0;
                    if (h.path) h.path[e] = 0.0;
                    if (h.D) h.D[e] = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        if (h.d_last) h.d_last[3 * e + a] = 0.f;
                        if (h.x_last) h.x_last[3 * e + a] = 0.f;
                        if (h.eH_last) h.eH_last[3 * e + a] = 0.f;
                        if (h.eV_last) h.eV_last[3 * e + a] = 0.f;
                    }
                }
                if (h.tri_path)
                    for (int bb = (hit ? 1 : 0); bb < p.bmax; ++bb) h.tri_path[e * p.bmax + bb] = -1;
            }
        } else {
            if (SRC == 0) {
                // first hits happen only here; a tile never spans two angles
                uint64_t m;
                const uint32_t pos = wave_alloc(p.rec_cnt + slot, hit, m);
                if (hit) r.rec = static_cast<int>(p.plans[slot].rec_base + pos);
            }
            if (hit) {
                const int e = r.rec;
                p.rec.r0[e] = make_float4(dlx, dly, dlz, __int_as_float(b.id));
                p.rec.r1[e] = make_float4(hlx, hly, hlz, __int_as_float(r.first));
                p.rec.r2[e] = make_float4(vlx, vly, vlz, __int_as_float(N | (flags << 8)));
                p.rec.D[e] = D;
            }
        }

        // ---- survivors to the next queue (one atomic per wave)
        uint64_t m;
        const uint32_t pos = wave_alloc(p.qout_cnt, cont, m);
        if (cont) {
            p.qout.s0[pos] = make_float4(r.ox, r.oy, r.oz, __int_as_float(r.prev));
            p.qout.s1[pos] = make_float4(r.dx, r.dy, r.dz, __int_as_float(r.first));
            p.qout.s2[pos] = make_float4(r.hx, r.hy, r.hz, __int_as_float(r.id));
            p.qout.s3[pos] = make_float4(r.vx, r.vy, r.vz, __int_as_float(r.meta));
            p.qout.s4[pos] = make_double2(r.P, r.comp);
            p.qout.s5[pos] = make_double2(r.kdo, __longlong_as_double(static_cast<long long>(r.rec)));
        }
    }

    // ---- statistics: one atomic per wave
    for (int off = 32; off >= 1; off >>= 1) {
        my_queries += __shfl_xor(my_queries, off);
        my_hits += __shfl_xor(my_hits, off);
        my_trapped += __shfl_xor(my_trapped, off);
    }
    if (lane == 0) {
        if (my_queries) atomicAdd(p.stat + ST_QUERIES, my_queries);
        if (my_hits) atomicAdd(p.stat + ST_HITS + p.bounce, my_hits);
        if (my_trapped) atomicAdd(p.stat + ST_TRAPPED, my_trapped);
    }
}

int g_blocks_cache = 0;

}  // namespace

int trace_block_threads() { return kBlock; }
int trace_stack_lds() { return kStackLds; }

int trace_persistent_blocks(sbr_ctx *ctx)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace<2>, kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 4;
    int blocks = ctx->prop.multiProcessorCount * per_cu;
    blocks = (blocks + 7) / 8 * 8;
    g_blocks_cache = blocks;
    return blocks;
}

static Params make_params(const TraceArgs &a, int bounce)
{
    Params p;
    p.nodes = a.bvh->nodes;
    p.tris = a.bvh->tris;
    p.nrm = a.bvh->nrm_slot;
    p.eps = a.bvh->eps;
    p.slack = static_cast<float>(1e-6 * a.bvh->diag) + 1e-30f;
    p.bmax = a.bmax;
    p.flags = a.flags;
    p.plans = a.plans;
    p.tile_base = a.tile_base;
    p.n_angles = a.n_angles;
    p.uo = a.rays ? a.rays->o : nullptr;
    p.ud = a.rays ? a.rays->d : nullptr;
    p.uh = a.rays ? a.rays->eH : nullptr;
    p.uv = a.rays ? a.rays->eV : nullptr;
    p.n_rays = a.n_rays;
    if (a.hits) p.hits = *a.hits;
    else p.hits = sbr_hits{};
    p.kx = a.k_hat[0];
    p.ky = a.k_hat[1];
    p.kz = a.k_hat[2];
    p.qin = a.q_in;
    p.qout = a.q_out;
    p.qin_cnt = a.q_cnt + (bounce - 1);
    p.qout_cnt = a.q_cnt + bounce;
    p.rec = a.rec;
    p.rec_cnt = a.rec_cnt;
    p.n_tiles = a.n_tiles;
    p.ctr = reinterpret_cast<uint32_t *>(a.stat + 8 + SBR_MAX_BOUNCES + 1) + 8 * bounce;
    p.stat = a.stat;
    p.spill = a.spill;
    p.bounce = bounce;
    p.user_sink = a.hits != nullptr;
    return p;
}

int launch_trace_grid(hipStream_t s, const TraceArgs &a, int bounce)
{
    Params p = make_params(a, bounce);
    p.user_sink = 0;
    k_trace<0><<<g_blocks_cache, kBlock, 0, s>>>(p);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_trace_rays(hipStream_t s, const TraceArgs &a)
{
    Params p = make_params(a, 1);
    p.user_sink = 1;
    p.n_tiles = (a.n_rays + kTileRays - 1) / kTileRays;
    k_trace<1><<<g_blocks_cache, kBlock, 0, s>>>(p);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_trace_queue(hipStream_t s, const TraceArgs &a, int bounce, bool user_sink)
{
    Params p = make_params(a, bounce);
    p.user_sink = user_sink ? 1 : 0;
    k_trace<2><<<g_blocks_cache, kBlock, 0, s>>>(p);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

}  // namespace sbr
