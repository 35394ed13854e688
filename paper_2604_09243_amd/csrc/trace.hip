// Multi-bounce ray transport (Algorithm 2) on gfx950.
//
// Two schedules share the traversal, the bounce update and the record sinks:
//
// STREAM (default): one persistent launch carries every ray through all of
//   its bounces in registers.  Between bounces the lanes whose ray ended are
//   refilled: a wave ballot of the idle lanes ranks them (mbcnt prefix count)
//   and idle lane k takes the k-th unused ray of the wave's current batch,
//   so the active rays stay packed into the wave without moving any ray
//   state.  A batch of 64-ray tiles is claimed with one atomic on one of
//   kClaimRanges counters, each on its own 256-byte line and owning a
//   contiguous range of tiles served by one XCD (a block's XCD is taken as
//   blockIdx % 8, the order in which workgroups are spread over the dies);
//   a wave whose range is empty steals, first within its XCD.
// WAVEFRONT: one launch per bounce.  Rays that hit and have bounces left are
//   compacted into the next bounce's queue with one atomic per wave (ballot
//   + prefix popcount); the next launch reads that queue.
//
// Rays of the incidence-angle grid (Eqs. L1-L3) are generated in-register:
// a 64-ray tile is a tile_w x (64 / tile_w) patch of the aperture.  Every hit overwrites the
// ray's record (one slot per ray), so a terminated ray's record holds its
// last hit; a ray that never hits writes an empty record.
//
// Closest hit: BVH2 traversal, both child boxes of a node per 64-byte fetch,
// nearer child first, the farther one on a per-lane stack that lives in LDS
// (spilling to a global array beyond kStackLds entries).  The loop is split
// in two phases per step: lanes descend through internal nodes until each
// holds a leaf (or is done), then the wave tests leaf triangles together;
// a leaf's triangles are read as whole 48-byte records with the next one
// prefetched.  The triangle test and the reflection arithmetic follow the
// float32 specification shared with the CPU oracle; this file is compiled
// with -ffp-contract=off, and fused multiply-adds are written explicitly
// only in the (conservative) box test.
#include <climits>
#include <cmath>
#include <mutex>
#include <string>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

constexpr int kBlock = 256;
#ifndef SBR_TRACE_STACK
#define SBR_TRACE_STACK 28
#endif
constexpr int kStackLds = SBR_TRACE_STACK;  // LDS stack entries per lane
#ifndef SBR_TRACE_SPILL_LDS
#define SBR_TRACE_SPILL_LDS 16
#endif
constexpr int kStackSpillLds = SBR_TRACE_SPILL_LDS;  // LDS part of the stack when deeper trees spill to global memory
// The closest hit is the minimum over every triangle of (t, id) among the
// hits that the float32 rule accepts (Moller-Trumbore conditions and the hit
// point inside its triangle's box widened by P).  The tree finds exactly that
// minimum:
//  * every BVH box contains the widened triangle boxes of its subtree plus a
//    guard G (SceneScale), which exceeds the float32 rounding of the hit point
//    and of the slab test below, so a box that holds an accepted hit point at
//    distance t' <= the best t so far always passes the test (entry <= t' <=
//    exit); no relative margin on t is needed;
//  * the rule is applied to every candidate that would improve the best hit
//    (with the triangle's record already in registers), so the best t is
//    always an accepted hit's and every box skipped against it held no
//    better accepted hit.
// Slab-test rounding: with ix = rcp(d) (1 ulp) and ox = fl(o ix), the value
// fma(b, ix, -ox) is within (3 2^-24 |b - o| + 2^-24 |o|) / |d| of (b - o) / d;
// the hit point fl(o + fl(t d)) is within 2^-24 (2 |x| + |o|) of o + t d.
// With every coordinate below M = X + obound that is less than 6 2^-24 M,
// under G = 8 2^-24 M.  Caller rays whose origin lies beyond obound get the
// difference as a per-ray widening of the slab values.
constexpr float kGuardUlps = 0x1p-21f;  // G / M
constexpr int kTileRays = 64;
// Five waves per SIMD: the LDS stack (28 entries x 256 lanes = 28 KB per
// block) lets five blocks share a CU, and the register allocator is held to
// 96 VGPRs (a few cold spills) so that all five fit; measured 10 % faster
// than four waves at 105 VGPRs.
#ifndef SBR_TRACE_WAVES_PER_SIMD
#define SBR_TRACE_WAVES_PER_SIMD 5  // occupancy floor handed to the register allocator
#endif
#define SBR_TRACE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(SBR_TRACE_WAVES_PER_SIMD)))
// Build with -DSBR_TRACE_COUNTERS to count traversal work into stat[2..7]:
// lane node visits, lane leaf visits, lane triangle tests, and wave-level
// trips of the internal-node loop, of the leaf step and of the bounce loop.
#ifdef SBR_TRACE_COUNTERS
#define SBR_COUNT(stmt) stmt
#else
#define SBR_COUNT(stmt)
#endif

struct Params {
    const BNode *nodes;
    const BNode4 *nodes4;  // the same tree four-wide (single-scene launches that walk it)
    const BTri *tris;
    const float4 *nrm;  // by slot
    float eps, pbox;    // caller rays: the scene's offset and the hit rule's P
    float obound;       // caller rays: origin coordinates up to this are covered by the BVH's guard
    int bmax;
    uint32_t flags;
    // grid source
    const AnglePlan *plans;
    const int64_t *tile_base;
    const uint8_t *mask;  // primary-ray mask of the plans (NULL: trace every ray)
    const int32_t *live;  // streaming schedule with a mask: the live tiles in order (NULL: every tile)
    const uint32_t *live_count;
    int n_angles;
    // caller source / sink
    const float *uo, *ud, *uh, *uv;
    int64_t n_rays;
    sbr_hits hits;
    double kx, ky, kz;
    // wavefront queues
    RayQueue qin, qout;
    const uint32_t *qin_cnt;
    uint32_t *qout_cnt;
    // records of the sweep (one slot per ray: plan.rec_base + ray id)
    Records rec;
    // misc
    int64_t n_tiles;
    uint32_t *ctr;  // kClaimRanges claim counters, kLineU32 apart
    unsigned long long *stat;
    int32_t *spill;
    int bounce;
    int user_sink;
    int tile_shift, claim_tiles, refill_min;  // launch parameters (sbr_tune)
    int packet;  // primary tiles may walk the tree as packets (binary tree, depth <= kPacketStack)
};

struct Ray {
    float ox, oy, oz, dx, dy, dz;
    float hx, hy, hz, vx, vy, vz;
    int prev, first, id, meta;  // meta = N | back << 7 | angle slot << 8
    double P, comp, kdo;
};

// Closest hit so far.  R is the traversal's arithmetic: float32 (the
// method) or float64 (the precision study SBR_OPT_FP64_TRAVERSE).
template <typename R>
struct BestT {
    R t;
    int id;
    int slot;
#ifdef SBR_TRACE_COUNTERS
    unsigned nodes, leaves, tris, wnode, wleaf;
#endif
};
using Best = BestT<float>;

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float minR(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double minR(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float maxR(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double maxR(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float rcpR(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpR(double x) { return 1.0 / x; }

__device__ __forceinline__ bool wave_leader()
{
    return static_cast<int>(threadIdx.x & 63) == __ffsll(static_cast<unsigned long long>(__ballot(1))) - 1;
}

template <typename R>
__device__ __forceinline__ bool tri_test(const BTri &tr, const Ray &r, R &t_out)
{
    const R e1x = tr.p1.x, e1y = tr.p1.y, e1z = tr.p1.z;
    const R e2x = tr.p2.x, e2y = tr.p2.y, e2z = tr.p2.z;
    const R dx = r.dx, dy = r.dy, dz = r.dz;
    const R px = dy * e2z - dz * e2y;
    const R py = dz * e2x - dx * e2z;
    const R pz = dx * e2y - dy * e2x;
    const R det = (e1x * px + e1y * py) + e1z * pz;
    if (det == R(0)) return false;
    const R sx = R(r.ox) - R(tr.p0.x), sy = R(r.oy) - R(tr.p0.y), sz = R(r.oz) - R(tr.p0.z);
    const R un = (sx * px + sy * py) + sz * pz;
    const R qx = sy * e1z - sz * e1y;
    const R qy = sz * e1x - sx * e1z;
    const R qz = sx * e1y - sy * e1x;
    const R vn = (dx * qx + dy * qy) + dz * qz;
    const R tn = (e2x * qx + e2y * qy) + e2z * qz;
    const R inv = R(1) / det;
    const R u = un * inv, v = vn * inv, t = tn * inv;
    t_out = t;
    return u >= R(0) && v >= R(0) && u + v <= R(1) && t > R(0) && t < R(INFINITY);
}

// The hit rule's box test: the hit point o + t d (the bounce update's
// point; float32 in the method) inside the triangle's box widened by P on
// every axis.
template <typename R>
__device__ __forceinline__ bool in_box(const BTri &tr, const Ray &r, R t, float P)
{
    const R x = R(r.ox) + t * R(r.dx), y = R(r.oy) + t * R(r.dy), z = R(r.oz) + t * R(r.dz);
    float lx, hx, ly, hy, lz, hz;
    spec_box_axis(tr.p0.x, tr.p1.x, tr.p2.x, P, lx, hx);
    spec_box_axis(tr.p0.y, tr.p1.y, tr.p2.y, P, ly, hy);
    spec_box_axis(tr.p0.z, tr.p1.z, tr.p2.z, P, lz, hz);
    return x >= R(lx) && x <= R(hx) && y >= R(ly) && y <= R(hy) && z >= R(lz) && z <= R(hz);
}

// Candidate triangle tr (leaf slot `slot`): it becomes the best hit when the
// float32 test accepts it, it is not the previous triangle, it improves
// (t, id), and its hit point passes the box rule.
template <typename R>
__device__ __forceinline__ void test_tri(const BTri &tr, int slot, const Ray &r, BestT<R> &b, float P)
{
    const int id = __float_as_int(tr.p0.w);
    R t;
    if (tri_test(tr, r, t) && id != r.prev && (t < b.t || (t == b.t && id < b.id)) && in_box(tr, r, t, P)) {
        b.t = t;
        b.id = id;
        b.slot = slot;
    }
}

constexpr int kEmpty = INT_MIN;  // never a valid node or leaf reference

// Stack of node/leaf references: kStackLds entries in LDS when the tree is
// shallow enough (SPILL = false), otherwise kStackSpillLds in LDS and the
// rest in a global spill array.
template <bool SPILL>
struct Stack {
    int *lst;        // this lane's LDS column (stride kBlock)
    int32_t *gst;    // this lane's spill column (stride gstride)
    int64_t gstride;
    __device__ __forceinline__ void push(int sp, int v)
    {
        if (!SPILL) {
            lst[sp * kBlock] = v;
        } else if (sp < kStackSpillLds) {
            lst[sp * kBlock] = v;
        } else {
            gst[(sp - kStackSpillLds) * gstride] = v;
        }
    }
    __device__ __forceinline__ int pop(int sp)
    {
        if (!SPILL) return lst[sp * kBlock];
        if (sp < kStackSpillLds) return lst[sp * kBlock];
        return gst[(sp - kStackSpillLds) * gstride];
    }
};

// Node and triangle records read through the scalar unit when every active
// lane of the wave wants the same one (coherent rays mostly do): the scalar
// loads bypass the vector memory pipeline, whose address unit otherwise
// limits the traversal.  Reads only.
typedef float sf4 __attribute__((ext_vector_type(4)));
typedef int si4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) sf4 *ScalarF4;
typedef const __attribute__((address_space(4))) si4 *ScalarI4;

__device__ __forceinline__ BNode node_scalar(const BNode *nodes, int i)
{
    const ScalarF4 q = (ScalarF4)(nodes + i);
    const sf4 a = q[0], b = q[1], c = q[2];
    const si4 ch = ((ScalarI4)(nodes + i))[3];
    BNode n;
    n.a = make_float4(a.x, a.y, a.z, a.w);
    n.b = make_float4(b.x, b.y, b.z, b.w);
    n.c = make_float4(c.x, c.y, c.z, c.w);
    n.ch = make_int4(ch.x, ch.y, ch.z, ch.w);
    return n;
}

struct ScalarTriLoader {
    const BTri *tris;
    __device__ __forceinline__ BTri operator[](int i) const
    {
        const ScalarF4 q = (ScalarF4)(tris + i);
        const sf4 a = q[0], b = q[1], c = q[2];
        BTri t;
        t.p0 = make_float4(a.x, a.y, a.z, a.w);
        t.p1 = make_float4(b.x, b.y, b.z, b.w);
        t.p2 = make_float4(c.x, c.y, c.z, c.w);
        return t;
    }
};

__device__ __forceinline__ bool wave_uniform(int v, int &v0)
{
    v0 = __builtin_amdgcn_readfirstlane(v);
    return __ballot(v != v0) == 0;
}

// The triangles [first, first + cnt) of a leaf, cnt <= 4, each 48-byte
// record loaded one test ahead.
template <typename TriPtr, typename R>
__device__ __forceinline__ void test_leaf_from(TriPtr tris, int first, int cnt, const Ray &r, BestT<R> &b, float P)
{
    SBR_COUNT(b.leaves += 1; b.tris += cnt);
    const BTri t0 = tris[first];
    BTri t1, t2, t3;
    if (cnt > 1) t1 = tris[first + 1];
    test_tri(t0, first, r, b, P);
    if (cnt > 2) t2 = tris[first + 2];
    if (cnt > 1) test_tri(t1, first + 1, r, b, P);
    if (cnt > 3) t3 = tris[first + 3];
    if (cnt > 2) test_tri(t2, first + 2, r, b, P);
    if (cnt > 3) test_tri(t3, first + 3, r, b, P);
}

// Leaf `code` (first triangle << 3 | count - 1).
template <typename R>
__device__ __forceinline__ void test_leaf(const Params &p, int code, const Ray &r, BestT<R> &b, float P)
{
    int c0;
    if (wave_uniform(code, c0))
        test_leaf_from(ScalarTriLoader{p.tris}, c0 >> 3, (c0 & 7) + 1, r, b, P);
    else
        test_leaf_from(p.tris, code >> 3, (code & 7) + 1, r, b, P);
}

// Entry and exit distances of the ray (inverse direction i, origin terms l
// for the low and h for the high planes of each axis) through both child
// boxes of node n, the exit clamped to tlim.
template <typename R>
__device__ __forceinline__ void node_boxes(const BNode &n, R ix, R iy, R iz, R lx, R ly, R lz, R hx, R hy, R hz,
                                           R tlim, R &t0, R &u0, R &t1, R &u1, int &cx, int &cy)
{
    // child 0: lo = (a.x, a.y, a.z), hi = (a.w, b.x, b.y)
    const R ax0 = fmaR(R(n.a.x), ix, -lx), ax1 = fmaR(R(n.a.w), ix, -hx);
    const R ay0 = fmaR(R(n.a.y), iy, -ly), ay1 = fmaR(R(n.b.x), iy, -hy);
    const R az0 = fmaR(R(n.a.z), iz, -lz), az1 = fmaR(R(n.b.y), iz, -hz);
    t0 = maxR(maxR(minR(ax0, ax1), minR(ay0, ay1)), maxR(minR(az0, az1), R(0)));
    u0 = minR(minR(maxR(ax0, ax1), maxR(ay0, ay1)), minR(maxR(az0, az1), tlim));
    // child 1: lo = (b.z, b.w, c.x), hi = (c.y, c.z, c.w)
    const R bx0 = fmaR(R(n.b.z), ix, -lx), bx1 = fmaR(R(n.c.y), ix, -hx);
    const R by0 = fmaR(R(n.b.w), iy, -ly), by1 = fmaR(R(n.c.z), iy, -hy);
    const R bz0 = fmaR(R(n.c.x), iz, -lz), bz1 = fmaR(R(n.c.w), iz, -hz);
    t1 = maxR(maxR(minR(bx0, bx1), minR(by0, by1)), maxR(minR(bz0, bz1), R(0)));
    u1 = minR(minR(maxR(bx0, bx1), maxR(by0, by1)), minR(maxR(bz0, bz1), tlim));
    cx = n.ch.x;
    cy = n.ch.y;
}

__device__ __forceinline__ BNode4 node4_scalar(const BNode4 *nodes, int i)
{
    const ScalarF4 q = (ScalarF4)(nodes + i);
    const sf4 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4], f = q[5];
    const si4 ch = ((ScalarI4)(nodes + i))[6];
    BNode4 n;
    n.lox = make_float4(a.x, a.y, a.z, a.w);
    n.hix = make_float4(b.x, b.y, b.z, b.w);
    n.loy = make_float4(c.x, c.y, c.z, c.w);
    n.hiy = make_float4(d.x, d.y, d.z, d.w);
    n.loz = make_float4(e.x, e.y, e.z, e.w);
    n.hiz = make_float4(f.x, f.y, f.z, f.w);
    n.ch = make_int4(ch.x, ch.y, ch.z, ch.w);
    n.m = make_int4(0, 0, 0, 0);
    return n;
}

__device__ __forceinline__ BNode4 node4_vector(const BNode4 *nodes, int i)
{
    const BNode4 *q = nodes + i;
    BNode4 n;
    n.lox = q->lox;
    n.hix = q->hix;
    n.loy = q->loy;
    n.hiy = q->hiy;
    n.loz = q->loz;
    n.hiz = q->hiz;
    n.ch = q->ch;
    n.m = make_int4(0, 0, 0, 0);
    return n;
}

// Entry/exit test of the four child boxes of node n (same slab arithmetic as
// node_boxes, exit clamped to tlim) -> the four sort keys.
template <typename R>
__device__ __forceinline__ void node4_keys(const BNode4 &n, R ix, R iy, R iz, R lx, R ly, R lz, R hx, R hy, R hz,
                                           R tlim, uint32_t &k0, uint32_t &k1, uint32_t &k2, uint32_t &k3)
{
    uint32_t k[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float bx0 = (&n.lox.x)[c], bx1 = (&n.hix.x)[c];
        const float by0 = (&n.loy.x)[c], by1 = (&n.hiy.x)[c];
        const float bz0 = (&n.loz.x)[c], bz1 = (&n.hiz.x)[c];
        const R ax0 = fmaR(R(bx0), ix, -lx), ax1 = fmaR(R(bx1), ix, -hx);
        const R ay0 = fmaR(R(by0), iy, -ly), ay1 = fmaR(R(by1), iy, -hy);
        const R az0 = fmaR(R(bz0), iz, -lz), az1 = fmaR(R(bz1), iz, -hz);
        const R tn = maxR(maxR(minR(ax0, ax1), minR(ay0, ay1)), maxR(minR(az0, az1), R(0)));
        const R tf = minR(minR(maxR(ax0, ax1), maxR(ay0, ay1)), minR(maxR(az0, az1), tlim));
        const int ref = (&n.ch.x)[c];
        // a passed child's key: its entry distance (>= 0, so the float bits
        // order as unsigned integers; float precision is enough for an order)
        // with its slot in the two low bits; ~0 for a missed or absent child
        k[c] = (tn <= tf && ref != kNoChild)
                   ? ((__float_as_uint(static_cast<float>(tn)) & ~3u) | static_cast<uint32_t>(c))
                   : ~0u;
    }
    k0 = k[0];
    k1 = k[1];
    k2 = k[2];
    k3 = k[3];
}

__device__ __forceinline__ void cswap(uint32_t &a, uint32_t &b)
{
    const uint32_t lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

__device__ __forceinline__ int pick_ref(const int4 &ch, uint32_t key)
{
    const uint32_t s = key & 3u;
    return s == 0 ? ch.x : s == 1 ? ch.y : s == 2 ? ch.z : ch.w;
}

// Whether rays come from and go to the caller (sbr_trace) rather than an
// angle grid (sweeps): U = 1 or 0 when the launch fixes it at compile time,
// U < 0 to read it from the launch parameters.
template <int U>
__device__ __forceinline__ bool user_rays(const Params &p)
{
    if constexpr (U >= 0) return U != 0;
    else return p.user_sink != 0;
}

// The scene a ray belongs to: its root node in the (possibly multi-scene)
// node array, its surface offset and the hit rule's P.
struct SceneRef {
    int root;
    float eps, pbox;
};

template <int U = -1>
__device__ __forceinline__ SceneRef scene_of(const Params &p, const Ray &r)
{
    if (user_rays<U>(p)) return SceneRef{0, p.eps, p.pbox};
    const AnglePlan &pl = p.plans[r.meta >> 8];
    return SceneRef{pl.root, pl.eps, pl.pbox};
}

// One traversal for the closest hit of ray r, skipping triangle r.prev.
// FAR: widen the slab values for an origin beyond the BVH guard's bound
// (caller rays).
template <bool SPILL, bool FAR, typename R, int W>
__device__ __forceinline__ BestT<R> traverse(const Params &p, const Ray &r, Stack<SPILL> st, const SceneRef sc)
{
    BestT<R> b;
    b.t = INFINITY;
    b.id = 0x7fffffff;
    b.slot = -1;
    SBR_COUNT(b.nodes = b.leaves = b.tris = b.wnode = b.wleaf = 0);
    const float tiny = 1e-20f;
    const R ddx = fabsf(r.dx) < tiny ? copysignf(tiny, r.dx) : r.dx;
    const R ddy = fabsf(r.dy) < tiny ? copysignf(tiny, r.dy) : r.dy;
    const R ddz = fabsf(r.dz) < tiny ? copysignf(tiny, r.dz) : r.dz;
    const R ix = rcpR(ddx), iy = rcpR(ddy), iz = rcpR(ddz);
    R lx = R(r.ox) * ix, ly = R(r.oy) * iy, lz = R(r.oz) * iz;
    R hx = lx, hy = ly, hz = lz;
    if constexpr (FAR) {
        // near planes earlier, far planes later by 8 2^-24 (|o| - obound) / |d|
        const R gx = R(kGuardUlps * fmaxf(fabsf(r.ox) - p.obound, 0.0f)) * ix;
        const R gy = R(kGuardUlps * fmaxf(fabsf(r.oy) - p.obound, 0.0f)) * iy;
        const R gz = R(kGuardUlps * fmaxf(fabsf(r.oz) - p.obound, 0.0f)) * iz;
        lx += gx; hx -= gx;
        ly += gy; hy -= gy;
        lz += gz; hz -= gz;
    }
    int sp = 0;
    int cur = W == 4 ? 0 : sc.root;  // the root is an internal node
    for (;;) {
        // phase 1: descend through internal nodes until a leaf (or nothing) is next
        while (W == 4 && cur >= 0) {
            SBR_COUNT(b.nodes += 1; if (wave_leader()) b.wnode += 1);
            int c0;
            const BNode4 nd = wave_uniform(cur, c0) ? node4_scalar(p.nodes4, c0) : node4_vector(p.nodes4, cur);
            uint32_t k0, k1, k2, k3;
            node4_keys(nd, ix, iy, iz, lx, ly, lz, hx, hy, hz, b.t, k0, k1, k2, k3);
            // nearest first: sort the four keys, go on with the nearest, push the rest far to near
            cswap(k0, k1);
            cswap(k2, k3);
            cswap(k0, k2);
            cswap(k1, k3);
            cswap(k1, k2);
            if (k0 == ~0u) {
                if (sp > 0) {
                    --sp;
                    cur = st.pop(sp);
                } else {
                    cur = kEmpty;
                }
            } else {
                if (k3 != ~0u) {
                    st.push(sp, pick_ref(nd.ch, k3));
                    ++sp;
                }
                if (k2 != ~0u) {
                    st.push(sp, pick_ref(nd.ch, k2));
                    ++sp;
                }
                if (k1 != ~0u) {
                    st.push(sp, pick_ref(nd.ch, k1));
                    ++sp;
                }
                cur = pick_ref(nd.ch, k0);
            }
        }
        while (W == 2 && cur >= 0) {
            SBR_COUNT(b.nodes += 1; if (wave_leader()) b.wnode += 1);
            R t0, u0, t1, u1;
            int cx, cy, c0;
            if (wave_uniform(cur, c0))
                node_boxes(node_scalar(p.nodes, c0), ix, iy, iz, lx, ly, lz, hx, hy, hz, b.t, t0, u0, t1, u1, cx, cy);
            else
                node_boxes(p.nodes[cur], ix, iy, iz, lx, ly, lz, hx, hy, hz, b.t, t0, u0, t1, u1, cx, cy);
            const bool h0 = t0 <= u0, h1 = t1 <= u1;
            if (h0 && h1) {
                int nr = cx, fr = cy;
                if (t1 < t0) {
                    nr = cy;
                    fr = cx;
                }
                st.push(sp, fr);
                ++sp;
                cur = nr;
            } else if (h0) {
                cur = cx;
            } else if (h1) {
                cur = cy;
            } else if (sp > 0) {
                --sp;
                cur = st.pop(sp);
            } else {
                cur = kEmpty;
            }
        }
        if (cur == kEmpty) break;
        // phase 2: the triangles of leaf `cur`
        SBR_COUNT(if (wave_leader()) b.wleaf += 1);
        test_leaf(p, ~cur, r, b, sc.pbox);
        if (sp > 0) {
            --sp;
            cur = st.pop(sp);
        } else {
            break;
        }
    }
    return b;
}

// Closest hits of the active lanes by one shared walk of the tree (a
// packet), for waves of parallel primary rays, which mostly want the same
// nodes: each lane tests every visited node's child boxes with its own ray
// (and its own best hit as the far limit), and the packet goes into a child
// when any lane's test passes, nearer child first by the lanes' vote.  A lane
// thus reaches every leaf its own traversal would, and may test extra
// triangles, which cannot change the minimum of (t, id) under the hit rule:
// the closest hit is the per-lane walk's.  Every node and triangle is read
// through the scalar unit.  The shared stack lives in two registers (lane k
// holds entry k, 128 entries; the launch checks the tree's depth), so the
// walk runs with every lane of the wave enabled: lanes without a ray
// (`act` false) take part in no vote and their results are not used.
constexpr int kPacketStack = 128;

__device__ __forceinline__ void packet_push(int &s0, int &s1, int &sp, int v, int lane)
{
    if (sp < 64) s0 = lane == sp ? v : s0;
    else s1 = lane == sp - 64 ? v : s1;
    ++sp;
}

__device__ __forceinline__ int packet_pop(int s0, int s1, int &sp)
{
    --sp;
    return sp < 64 ? __builtin_amdgcn_readlane(s0, sp) : __builtin_amdgcn_readlane(s1, sp - 64);
}

template <typename R>
__device__ __forceinline__ BestT<R> traverse_packet(const Params &p, const Ray &r, const SceneRef sc, bool act,
                                                    int first)
{
    BestT<R> b;
    b.t = INFINITY;
    b.id = 0x7fffffff;
    b.slot = -1;
    SBR_COUNT(b.nodes = b.leaves = b.tris = b.wnode = b.wleaf = 0);
    const float tiny = 1e-20f;
    const R ddx = fabsf(r.dx) < tiny ? copysignf(tiny, r.dx) : r.dx;
    const R ddy = fabsf(r.dy) < tiny ? copysignf(tiny, r.dy) : r.dy;
    const R ddz = fabsf(r.dz) < tiny ? copysignf(tiny, r.dz) : r.dz;
    const R ix = rcpR(ddx), iy = rcpR(ddy), iz = rcpR(ddz);
    const R lx = R(r.ox) * ix, ly = R(r.oy) * iy, lz = R(r.oz) * iz;
    const int lane = threadIdx.x & 63;
    int s0 = 0, s1 = 0, sp = 0;
    int cur = __builtin_amdgcn_readlane(sc.root, first);  // the scene of the first active lane: one per wave
    for (;;) {
        while (cur >= 0) {
            SBR_COUNT(b.nodes += 1; if (wave_leader()) b.wnode += 1);
            R t0, u0, t1, u1;
            int cx, cy;
            node_boxes(node_scalar(p.nodes, cur), ix, iy, iz, lx, ly, lz, lx, ly, lz, b.t, t0, u0, t1, u1, cx, cy);
            const bool h0 = act && t0 <= u0, h1 = act && t1 <= u1;
            const uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
            if (m0 && m1) {
                const int both = __popcll(m0 & m1), c1first = __popcll(__ballot(h0 && h1 && t1 < t0));
                const bool swap = 2 * c1first > both;
                packet_push(s0, s1, sp, swap ? cx : cy, lane);
                cur = swap ? cy : cx;
            } else if (m0) {
                cur = cx;
            } else if (m1) {
                cur = cy;
            } else if (sp > 0) {
                cur = packet_pop(s0, s1, sp);
            } else {
                cur = kEmpty;
            }
        }
        if (cur == kEmpty) break;
        SBR_COUNT(if (wave_leader()) b.wleaf += 1);
        test_leaf_from(ScalarTriLoader{p.tris}, (~cur) >> 3, ((~cur) & 7) + 1, r, b, sc.pbox);
        if (sp > 0) cur = packet_pop(s0, s1, sp);
        else break;
    }
    return b;
}

// Whether the lanes holding a ray (`act`; the first of them `first`) hold
// parallel primary rays of one scene: those walk the tree as a packet.
// Called with every lane of the wave enabled.
__device__ __forceinline__ bool primary_wave(const Ray &r, const SceneRef &sc, bool act, int first)
{
    const int dx = __builtin_amdgcn_readlane(__float_as_int(r.dx), first);
    const int dy = __builtin_amdgcn_readlane(__float_as_int(r.dy), first);
    const int dz = __builtin_amdgcn_readlane(__float_as_int(r.dz), first);
    const int root = __builtin_amdgcn_readlane(sc.root, first);
    return __ballot(act && ((r.meta & 127) != 0 || __float_as_int(r.dx) != dx || __float_as_int(r.dy) != dy ||
                            __float_as_int(r.dz) != dz || sc.root != root)) == 0;
}

// Closest hit of ray r under the hit rule: one traversal that applies the
// rule to every candidate that would improve the best hit.
template <bool SPILL, bool FAR = false, typename R = float, int W = 2>
__device__ BestT<R> closest(const Params &p, const Ray &r, Stack<SPILL> st, const SceneRef sc)
{
    return traverse<SPILL, FAR, R, W>(p, r, st, sc);
}

struct K3 {
    double x, y, z;
};

__device__ __forceinline__ double dotk(const K3 &k, float x, float y, float z)
{
    return (k.x * static_cast<double>(x) + k.y * static_cast<double>(y)) + k.z * static_cast<double>(z);
}

__device__ __forceinline__ K3 plan_k(const AnglePlan &pl) { return K3{pl.k[0], pl.k[1], pl.k[2]}; }

// k . o of a fresh ray's origin: float64, or float32 in the precision study.
__device__ __forceinline__ double kdot0(const Params &p, const K3 &k, const Ray &r)
{
    if (!(p.flags & SBR_OPT_FP32_PATH)) return dotk(k, r.ox, r.oy, r.oz);
    const float kx = static_cast<float>(k.x), ky = static_cast<float>(k.y), kz = static_cast<float>(k.z);
    return static_cast<double>((kx * r.ox + ky * r.oy) + kz * r.oz);
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = threadIdx.x & 63;
    return (1ull << lane) - 1ull;
}

// Claims a batch of up to `batch` units from kClaimRanges contiguous ranges
// of [0, n_units), each with its own counter line; `home` = blockIdx %
// kClaimRanges, so a range serves one XCD (home % 8) and a few of its CUs,
// and every counter is shared by few waves.  When the home range is
// exhausted the wave steals: first from the other ranges of its XCD, then
// from the other XCDs'.  Returns the first unit and sets *end, or returns -1
// when every range is exhausted.
__device__ __forceinline__ int64_t claim(uint32_t *ctr, int64_t n_units, int home, int batch, int64_t *end)
{
    constexpr int kPerXcd = kClaimRanges / 8;
    for (int x = 0; x < 8; ++x) {
        for (int y = 0; y < kPerXcd; ++y) {
            const int c = ((home + x) & 7) + 8 * ((home / 8 + y) % kPerXcd);
            const int64_t lo = n_units * c / kClaimRanges, hi = n_units * (c + 1) / kClaimRanges;
            if (hi <= lo) continue;
            const uint32_t t = atomicAdd(&ctr[c * kLineU32], static_cast<uint32_t>(batch));
            if (lo + static_cast<int64_t>(t) < hi) {
                *end = min(lo + static_cast<int64_t>(t) + batch, hi);
                return lo + t;
            }
        }
    }
    return -1;
}

// Wave-aggregated atomic add: every lane with `want` gets a distinct slot
// from *ctr (consecutive within the wave, in lane order).
__device__ __forceinline__ uint32_t wave_alloc(uint32_t *ctr, bool want)
{
    const uint64_t m = __ballot(want);
    uint32_t base = 0;
    if (m) {
        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
        if ((threadIdx.x & 63) == leader) base = atomicAdd(ctr, static_cast<uint32_t>(__popcll(m)));
        base = __shfl(base, leader);
    }
    return base + static_cast<uint32_t>(__popcll(m & lanemask_lt()));
}

// The angle whose tiles hold `tile`, searched in angles [lo, hi).
__device__ __forceinline__ int find_angle(const Params &p, int64_t tile, int lo, int hi)
{
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (p.tile_base[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

typedef const __attribute__((address_space(4))) int64_t *ScalarI64;

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    return static_cast<int64_t>(static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(
                                    static_cast<int>(v >> 32))))
                                << 32) |
           static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v)));
}

// The angle of a wave-uniform tile through the scalar unit: a galloping
// search of tile_base up from angle `hint` when the tile lies at or past
// it, else a search below it.
__device__ __forceinline__ int find_angle_scalar(const Params &p, int64_t tile, int hint)
{
    const ScalarI64 tb = (ScalarI64)p.tile_base;
    const int n = p.n_angles;
    int lo = 0, hi = hint;
    if (tb[hint] <= tile) {  // tb[lo] <= tile < tb[hi], tb[n] above every tile
        lo = hint;
        hi = hint + 1;
        for (int step = 1; hi < n && tb[hi] <= tile; step *= 2) {
            lo = hi;
            hi = min(lo + step, n);
        }
    }
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tb[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Angles of the first and the last tile of a claimed batch; the search
// starts from the previous batch's last angle (claims from one range
// advance).  Every later lookup in the batch searches only between them
// (usually a single angle).
__device__ __forceinline__ void batch_angles(const Params &p, int64_t first, int64_t last, int &a_lo, int &a_hi)
{
    const int hint = __builtin_amdgcn_readfirstlane(a_hi);
    a_lo = find_angle_scalar(p, uniform64(first), hint);
    a_hi = find_angle_scalar(p, uniform64(last), a_lo);
}

typedef const __attribute__((address_space(4))) int32_t *ScalarI32;

// Position q of the angle grid (tile = q / 64, position in the tile's
// tile_w-wide patch = q % 64) -> kGridRay with a fresh ray in r; kGridNone
// if q lies outside the angle's N_u x N_v grid; kGridMasked if the ray's
// mask cell is empty: no leaf box can be hit, so the ray is a miss without
// traversal (no record, as for a miss).
constexpr int kGridNone = 0, kGridRay = 1, kGridMasked = 2;

__device__ __forceinline__ int grid_ray(const Params &p, int64_t q, Ray &r, int a_lo, int a_hi)
{
    const int64_t tile = q >> 6;
    const int k = static_cast<int>(q & 63);
    const int lo = find_angle(p, tile, a_lo, a_hi + 1);
    const AnglePlan &pl = p.plans[lo];
    const uint32_t t = static_cast<uint32_t>(tile - pl.tile_base);  // < tu tv < 2^32 (an angle holds < 2^31 rays)
    const int tw = 1 << p.tile_shift;
    const int i = static_cast<int>(t % static_cast<uint32_t>(pl.tu)) * tw + (k & (tw - 1));
    const int j = static_cast<int>(t / static_cast<uint32_t>(pl.tu)) * (kTileRays >> p.tile_shift) + (k >> p.tile_shift);
    if (i >= pl.nu || j >= pl.nv) return kGridNone;
    if (p.mask && p.mask[pl.mask_base + static_cast<int64_t>(j >> kMaskShift) * pl.mcu + (i >> kMaskShift)] == 0)
        return kGridMasked;  // no record (its byte stays 0)
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
    r.meta = lo << 8;
    r.P = 0.0;
    r.comp = 0.0;
    r.kdo = kdot0(p, plan_k(pl), r);
    return kGridRay;
}

// A whole tile whose mask cells are all empty: its in-grid positions (every
// one a miss without traversal, as grid_ray would find ray by ray), else -1.
__device__ __forceinline__ int masked_tile(const Params &p, int64_t tile, int a_lo, int a_hi)
{
    const int lo = find_angle(p, tile, a_lo, a_hi + 1);
    const AnglePlan &pl = p.plans[lo];
    const uint32_t t = static_cast<uint32_t>(tile - pl.tile_base);
    const int tw = 1 << p.tile_shift, th = kTileRays >> p.tile_shift;
    const int i0 = static_cast<int>(t % static_cast<uint32_t>(pl.tu)) * tw;
    const int j0 = static_cast<int>(t / static_cast<uint32_t>(pl.tu)) * th;
    const int i1 = min(i0 + tw, pl.nu), j1 = min(j0 + th, pl.nv);  // i0 < nu, j0 < nv for every tile of the angle
    const uint8_t *m = p.mask + pl.mask_base;
    for (int cj = j0 >> kMaskShift; cj <= (j1 - 1) >> kMaskShift; ++cj)
        for (int ci = i0 >> kMaskShift; ci <= (i1 - 1) >> kMaskShift; ++ci)
            if (m[static_cast<int64_t>(cj) * pl.mcu + ci]) return -1;
    return (i1 - i0) * (j1 - j0);
}

// Ray e of the caller's arrays; false if e >= n_rays.
__device__ __forceinline__ bool user_ray(const Params &p, int64_t e, Ray &r)
{
    if (e >= p.n_rays) return false;
    r.ox = p.uo[3 * e];
    r.oy = p.uo[3 * e + 1];
    r.oz = p.uo[3 * e + 2];
    r.dx = p.ud[3 * e];
    r.dy = p.ud[3 * e + 1];
    r.dz = p.ud[3 * e + 2];
    r.hx = p.uh[3 * e];
    r.hy = p.uh[3 * e + 1];
    r.hz = p.uh[3 * e + 2];
    r.vx = p.uv[3 * e];
    r.vy = p.uv[3 * e + 1];
    r.vz = p.uv[3 * e + 2];
    r.prev = -1;
    r.first = -1;
    r.id = static_cast<int>(e);
    r.meta = 0;
    r.P = 0.0;
    r.comp = 0.0;
    r.kdo = kdot0(p, K3{p.kx, p.ky, p.kz}, r);
    if (p.hits.tri_path)
        for (int b = 0; b < p.bmax; ++b) p.hits.tri_path[e * p.bmax + b] = -1;
    return true;
}

struct Last {
    float dlx, dly, dlz, xlx, xly, xlz, hlx, hly, hlz, vlx, vly, vlz;
    double D;
    int flags;
};

// Algorithm 2 bookkeeping for a hit b of ray r, then the specular
// reflection of the direction and of both field vectors, and the new origin
// eps off the surface on the side the ray came from.  Returns whether the
// ray has bounces left.
template <typename R>
__device__ __forceinline__ bool bounce(const Params &p, Ray &r, const BestT<R> &b, const K3 &kv, const float eps,
                                       Last &L)
{
    const R tr = b.t;
    L.xlx = static_cast<float>(R(r.ox) + tr * R(r.dx));
    L.xly = static_cast<float>(R(r.oy) + tr * R(r.dy));
    L.xlz = static_cast<float>(R(r.oz) + tr * R(r.dz));
    const float t = static_cast<float>(tr);
    int N = r.meta & 127;
    const bool f32 = (p.flags & SBR_OPT_FP32_PATH) != 0;  // precision study: path, offset term and D in float32
    if (!f32) {
        r.P = r.P + static_cast<double>(tr);
        if (N >= 1 && !(p.flags & SBR_OPT_PAPER_PATH)) r.P = r.P + r.comp;
    } else {
        float P32 = static_cast<float>(r.P) + t;
        if (N >= 1 && !(p.flags & SBR_OPT_PAPER_PATH)) P32 = P32 + static_cast<float>(r.comp);
        r.P = static_cast<double>(P32);
    }
    N += 1;
    if (N == 1) r.first = b.id;
    L.dlx = r.dx;
    L.dly = r.dy;
    L.dlz = r.dz;
    L.hlx = r.hx;
    L.hly = r.hy;
    L.hlz = r.hz;
    L.vlx = r.vx;
    L.vly = r.vy;
    L.vlz = r.vz;
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
    r.ox = L.xlx + eps * nfx;
    r.oy = L.xly + eps * nfy;
    r.oz = L.xlz + eps * nfz;
    if (!f32) {
        r.comp = static_cast<double>(eps) * ((static_cast<double>(nfx) * r.dx + static_cast<double>(nfy) * r.dy) +
                                             static_cast<double>(nfz) * r.dz);
    } else {
        r.comp = static_cast<double>(eps * ((nfx * r.dx + nfy * r.dy) + nfz * r.dz));
    }
    r.prev = b.id;
    r.meta = (r.meta & ~0xff) | N | (back ? 128 : 0);
    if (!f32) {
        L.D = (r.kdo + r.P) + dotk(kv, L.xlx, L.xly, L.xlz);
    } else {
        const float kx = static_cast<float>(kv.x), ky = static_cast<float>(kv.y), kz = static_cast<float>(kv.z);
        L.D = static_cast<double>((static_cast<float>(r.kdo) + static_cast<float>(r.P)) +
                                  ((kx * L.xlx + ky * L.xly) + kz * L.xlz));
    }
    L.flags = SBR_REC_VALID | (back ? SBR_REC_BACK_LAST : 0);
    return N < p.bmax;
}

// Slot e of the sweep records holds a record (the ray's own byte).
__device__ __forceinline__ void mark_record(const Params &p, int64_t e) { p.rec.held[e] = 1; }

template <int U = -1, typename R = float>
__device__ __forceinline__ void sink_hit(const Params &p, const Ray &r, const BestT<R> &b, const Last &L)
{
    const int N = r.meta & 127;
    if (user_rays<U>(p)) {
        const sbr_hits &h = p.hits;
        const int64_t e = r.id;
        if (h.n_bounce) h.n_bounce[e] = N;
        if (h.tri_first) h.tri_first[e] = r.first;
        if (h.tri_last) h.tri_last[e] = b.id;
        if (h.flags) h.flags[e] = L.flags;
        if (h.path) h.path[e] = r.P;
        if (h.D) h.D[e] = L.D;
        if (h.d_last) { h.d_last[3 * e] = L.dlx; h.d_last[3 * e + 1] = L.dly; h.d_last[3 * e + 2] = L.dlz; }
        if (h.x_last) { h.x_last[3 * e] = L.xlx; h.x_last[3 * e + 1] = L.xly; h.x_last[3 * e + 2] = L.xlz; }
        if (h.eH_last) { h.eH_last[3 * e] = L.hlx; h.eH_last[3 * e + 1] = L.hly; h.eH_last[3 * e + 2] = L.hlz; }
        if (h.eV_last) { h.eV_last[3 * e] = L.vlx; h.eV_last[3 * e + 1] = L.vly; h.eV_last[3 * e + 2] = L.vlz; }
        if (h.tri_path) h.tri_path[e * p.bmax + (N - 1)] = b.id;
    } else {
        const int64_t e = p.plans[r.meta >> 8].rec_base + r.id;
        Rec &q = p.rec.rec[e];
        q.r0 = make_float4(L.dlx, L.dly, L.dlz, __int_as_float(b.slot));  // the triangle's leaf slot
        q.r1 = make_float4(L.hlx, L.hly, L.hlz, __int_as_float(r.first));
        q.r2 = make_float4(L.vlx, L.vly, L.vlz, __int_as_float(N | (L.flags << 8)));
        q.D = make_double2(L.D, 0.0);
        if (N == 1) mark_record(p, e);
    }
}

// The sweep record of ray r from its last hit (the hit triangle's leaf slot
// slot_last, bookkeeping L, record flags fl), written once when the ray
// ends, and only when it enters the PO sum (a trapped ray dropped by
// SBR_OPT_DROP_TRAPPED writes nothing).  The slot, not the triangle id:
// the PO stage reads the normal in leaf order, where the normals of
// neighbouring rays share cache lines.
__device__ __forceinline__ void sink_record(const Params &p, const Ray &r, int slot_last, const Last &L, int fl)
{
    if (!(fl & SBR_REC_VALID)) return;
    const int N = r.meta & 127;
    const int64_t e = p.plans[r.meta >> 8].rec_base + r.id;
    Rec &q = p.rec.rec[e];
    q.r0 = make_float4(L.dlx, L.dly, L.dlz, __int_as_float(slot_last));
    q.r1 = make_float4(L.hlx, L.hly, L.hlz, __int_as_float(r.first));
    q.r2 = make_float4(L.vlx, L.vly, L.vlz, __int_as_float(N | (fl << 8)));
    q.D = make_double2(L.D, 0.0);
    mark_record(p, e);
}

// A ray whose first query missed: an empty record.
template <int U = -1>
__device__ __forceinline__ void sink_miss(const Params &p, const Ray &r)
{
    if (user_rays<U>(p)) {
        const sbr_hits &h = p.hits;
        const int64_t e = r.id;
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
    // sweep records: nothing (the slot's byte stays 0)
}

template <int U = -1>
__device__ __forceinline__ void flag_trapped(const Params &p, const Ray &r)
{
    const int N = r.meta & 127;
    if (user_rays<U>(p)) {
        if (p.hits.flags) p.hits.flags[r.id] = (p.hits.flags[r.id] | SBR_REC_TRAPPED) & ~SBR_REC_VALID;
    } else {
        const int64_t e = p.plans[r.meta >> 8].rec_base + r.id;
        float4 v = p.rec.rec[e].r2;
        const int fl = ((__float_as_int(v.w) >> 8) | SBR_REC_TRAPPED) & ~SBR_REC_VALID;
        v.w = __int_as_float(N | (fl << 8));
        p.rec.rec[e].r2 = v;
    }
}

template <int U = -1>
__device__ __forceinline__ K3 kvec(const Params &p, const Ray &r)
{
    if (user_rays<U>(p)) return K3{p.kx, p.ky, p.kz};
    return plan_k(p.plans[r.meta >> 8]);
}

// Per-block counters in LDS, flushed with one global atomic each at the end.
struct BlockStats {
    unsigned int queries, trapped, masked;
    unsigned int hits[SBR_MAX_BOUNCES + 1];
    unsigned long long diag[6];
};

template <typename R>
__device__ __forceinline__ void count_query(BlockStats &bs, const BestT<R> &b)
{
#ifdef SBR_TRACE_COUNTERS
    atomicAdd(&bs.diag[0], static_cast<unsigned long long>(b.nodes));
    atomicAdd(&bs.diag[1], static_cast<unsigned long long>(b.leaves));
    atomicAdd(&bs.diag[2], static_cast<unsigned long long>(b.tris));
    atomicAdd(&bs.diag[3], static_cast<unsigned long long>(b.wnode));
    atomicAdd(&bs.diag[4], static_cast<unsigned long long>(b.wleaf));
#endif
}

__device__ __forceinline__ void flush_stats(const Params &p, BlockStats &bs)
{
    __syncthreads();
    const int t = threadIdx.x;
    if (t == 0 && bs.queries) atomicAdd(p.stat + 0, static_cast<unsigned long long>(bs.queries));
    if (t == 1 && bs.trapped) atomicAdd(p.stat + 1, static_cast<unsigned long long>(bs.trapped));
    if (t == 2 && bs.masked) atomicAdd(p.stat + kStatMasked, static_cast<unsigned long long>(bs.masked));
    if (t >= 8 && t <= 8 + SBR_MAX_BOUNCES && bs.hits[t - 8])
        atomicAdd(p.stat + t, static_cast<unsigned long long>(bs.hits[t - 8]));
#ifdef SBR_TRACE_COUNTERS
    if (t >= 2 && t < 8 && bs.diag[t - 2]) atomicAdd(p.stat + t, bs.diag[t - 2]);
#endif
}

__device__ __forceinline__ void init_stats(BlockStats &bs)
{
    const int t = threadIdx.x;
    if (t == 0) {
        bs.queries = 0;
        bs.trapped = 0;
        bs.masked = 0;
    }
    if (t <= SBR_MAX_BOUNCES) bs.hits[t] = 0;
    if (t < 6) bs.diag[t] = 0;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// STREAM schedule
// ---------------------------------------------------------------------------
// (The float64 study variant holds twice the registers of the traversal
// state: three waves per SIMD instead of spilling.)
// W: node width of the tree walked (2: BNode, 4: BNode4).
template <int SRC, bool SPILL, typename R = float, int W = 2>  // SRC: 0 = angle grid, 1 = caller rays; R: see BestT
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 3 : SBR_TRACE_WAVES_PER_SIMD))) void k_stream(Params p)
{
    constexpr int kUser = SRC == 1;  // caller rays in, hit arrays out (else an angle grid and sweep records)
    __shared__ int lds_stack[(SPILL ? kStackSpillLds : kStackLds) * kBlock];
    __shared__ BlockStats bs;
    init_stats(bs);
    Stack<SPILL> st;
    st.lst = lds_stack + threadIdx.x;
    st.gstride = static_cast<int64_t>(gridDim.x) * kBlock;
    st.gst = p.spill + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int home = blockIdx.x % kClaimRanges;  // this block's claim range (on XCD blockIdx % 8)
    const uint64_t lt = lanemask_lt();
    // units: tiles of the angle grid (positions of the live-tile list when
    // the mask made one), or 64-ray groups of caller rays
    const int64_t n_units = SRC == 0 ? (p.live ? static_cast<int64_t>(*p.live_count) : p.n_tiles)
                                     : (p.n_rays + kTileRays - 1) / kTileRays;
    int64_t pos = 0, end = 0;  // wave-uniform: unused positions [pos, end) of the claimed batch
    int a_lo = 0, a_hi = 0;    // wave-uniform: angles spanned by the claimed batch
    bool src_done = false;
    bool has = false;
    Ray r;
    // the last hit of the lane's ray: a sweep record is written once, when the
    // ray ends (caller rays are written at every hit)
    Last L;
    int slot_last = -1;

    for (;;) {
        // ---- refill: idle lanes, ranked by a ballot prefix count, take the next positions
        for (;;) {
            const uint64_t idle = __ballot(!has);
            if (idle == 0 || src_done) break;
            if (__popcll(idle) < p.refill_min && idle != __ballot(1)) break;
            if (pos >= end) {
                int64_t u = -1, e = 0;
                if (lane == 0) u = claim(p.ctr, n_units, home, p.claim_tiles, &e);
                u = __shfl(u, 0);
                e = __shfl(e, 0);
                if (u < 0) {
                    src_done = true;
                    break;
                }
                pos = u * kTileRays;
                end = e * kTileRays;
                if (SRC == 0) {
                    int64_t first = u, last = e - 1;
                    if (p.live) {
                        first = ((ScalarI32)p.live)[uniform64(first)];
                        last = ((ScalarI32)p.live)[uniform64(last)];
                    }
                    batch_angles(p, first, last, a_lo, a_hi);
                }
            }
            const int64_t q = pos + static_cast<int64_t>(__popcll(idle & lt));
            if (!has && q < end) {
                if (SRC == 0) {
                    // position q of the list: ray q % 64 of live tile q / 64
                    const int64_t qg = p.live ? (static_cast<int64_t>(p.live[q >> 6]) << 6) | (q & 63) : q;
                    const int g = grid_ray(p, qg, r, a_lo, a_hi);
                    has = g == kGridRay;
                    if (g == kGridMasked) {
                        atomicAdd(&bs.queries, 1u);
                        atomicAdd(&bs.masked, 1u);
                    }
                } else {
                    has = user_ray(p, q, r);
                }
            }
            pos = min(pos + static_cast<int64_t>(__popcll(idle)), end);
        }
        if (__ballot(has) == 0) break;

        // ---- one bounce for every lane holding a ray
        BestT<R> b;
        b.slot = -1;
        SceneRef sc{0, 0.f, 0.f};
        if (has) sc = scene_of<kUser>(p, r);
        // (every lane of the wave is enabled here)
        const int first = __ffsll(static_cast<unsigned long long>(__ballot(has))) - 1;
        if (SRC == 0 && W == 2 && sizeof(R) == 4 && p.packet && primary_wave(r, sc, has, first)) {
            const BestT<R> bp = traverse_packet<R>(p, r, sc, has, first);
            if (has) b = bp;
        } else if (has) {
            b = closest<SPILL, SRC == 1, R, W>(p, r, st, sc);
        }
        if (has) atomicAdd(&bs.queries, 1u);
        SBR_COUNT(if (has) count_query(bs, b); if (threadIdx.x % 64 == 0) atomicAdd(&bs.diag[5], 1ull));
        if (has) {
            if (b.slot >= 0) {
                const K3 kv = kvec<kUser>(p, r);
                const bool cont = bounce(p, r, b, kv, sc.eps, L);
                slot_last = b.slot;
                atomicAdd(&bs.hits[r.meta & 127], 1u);
                if (kUser) sink_hit<kUser>(p, r, b, L);  // caller rays: every hit (the path of ids)
                if (!cont) {
                    int fl = L.flags;
                    if (p.flags & SBR_OPT_DROP_TRAPPED) {
                        const BestT<R> b2 = closest<SPILL, SRC == 1, R, W>(p, r, st, sc);
                        atomicAdd(&bs.queries, 1u);
                        if (b2.slot >= 0) {  // trapped: flagged and dropped from the PO sum
                            if (kUser) flag_trapped<kUser>(p, r);
                            fl = (fl | SBR_REC_TRAPPED) & ~SBR_REC_VALID;
                            atomicAdd(&bs.trapped, 1u);
                        }
                    }
                    if (!kUser) sink_record(p, r, slot_last, L, fl);
                    has = false;
                }
            } else {
                if ((r.meta & 127) == 0) sink_miss<kUser>(p, r);
                else if (!kUser) sink_record(p, r, slot_last, L, L.flags);
                has = false;
            }
        }
    }
    flush_stats(p, bs);
}

// ---------------------------------------------------------------------------
// WAVEFRONT schedule (one launch per bounce, queue between launches)
// ---------------------------------------------------------------------------
template <int SRC, bool SPILL>  // SRC: 0 = angle grid, 1 = caller rays, 2 = queue
__global__ __launch_bounds__(kBlock) SBR_TRACE_OCCUPANCY void k_wave(Params p)
{
    __shared__ int lds_stack[(SPILL ? kStackSpillLds : kStackLds) * kBlock];
    __shared__ BlockStats bs;
    init_stats(bs);
    Stack<SPILL> st;
    st.lst = lds_stack + threadIdx.x;
    st.gstride = static_cast<int64_t>(gridDim.x) * kBlock;
    st.gst = p.spill + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int home = blockIdx.x % kClaimRanges;  // this block's claim range (on XCD blockIdx % 8)
    int64_t n_units = SRC == 0 ? p.n_tiles : (p.n_rays + kTileRays - 1) / kTileRays;
    int64_t n_in = 0;
    if (SRC == 2) {
        n_in = *p.qin_cnt;
        n_units = (n_in + kTileRays - 1) / kTileRays;
    }
    int64_t tile = 0, tend = 0;  // wave-uniform claimed batch of tiles
    int a_lo = 0, a_hi = 0;
    for (;;) {
        if (tile >= tend) {
            int64_t u = -1, e = 0;
            if (lane == 0) u = claim(p.ctr, n_units, home, p.claim_tiles, &e);
            u = __shfl(u, 0);
            e = __shfl(e, 0);
            if (u < 0) break;
            tile = u;
            tend = e;
            if (SRC == 0) batch_angles(p, u, e - 1, a_lo, a_hi);
        }
        const int64_t q = tile * kTileRays + lane;
        ++tile;
        Ray r;
        bool active;
        if (SRC == 0) {
            const int g = grid_ray(p, q, r, a_lo, a_hi);
            active = g == kGridRay;
            if (g == kGridMasked) {
                atomicAdd(&bs.queries, 1u);
                atomicAdd(&bs.masked, 1u);
            }
        } else if (SRC == 1) {
            active = user_ray(p, q, r);
        } else {
            active = q < n_in;
            const int64_t e = active ? q : 0;
            const float4 s0 = p.qin.s0[e], s1 = p.qin.s1[e], s2 = p.qin.s2[e], s3 = p.qin.s3[e];
            const double2 s4 = p.qin.s4[e], s5 = p.qin.s5[e];
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
        }
        Best b;
        b.slot = -1;
        SceneRef sc{0, 0.f, 0.f};
        if (active) sc = scene_of(p, r);
        if (active) b = closest<SPILL, SRC == 1>(p, r, st, sc);
        if (active) atomicAdd(&bs.queries, 1u);
        SBR_COUNT(if (active) count_query(bs, b); if (threadIdx.x % 64 == 0) atomicAdd(&bs.diag[5], 1ull));
        bool cont = false;
        if (active) {
            if (b.slot >= 0) {
                const K3 kv = kvec(p, r);
                Last L;
                cont = bounce(p, r, b, kv, sc.eps, L);
                atomicAdd(&bs.hits[r.meta & 127], 1u);
                sink_hit(p, r, b, L);
                if (!cont && (p.flags & SBR_OPT_DROP_TRAPPED)) {
                    const Best b2 = closest<SPILL, SRC == 1>(p, r, st, sc);
                    atomicAdd(&bs.queries, 1u);
                    if (b2.slot >= 0) {
                        flag_trapped(p, r);
                        atomicAdd(&bs.trapped, 1u);
                    }
                }
            } else if ((r.meta & 127) == 0) {
                sink_miss(p, r);
            }
        }
        const uint32_t pos = wave_alloc(p.qout_cnt, cont);
        if (cont) {
            p.qout.s0[pos] = make_float4(r.ox, r.oy, r.oz, __int_as_float(r.prev));
            p.qout.s1[pos] = make_float4(r.dx, r.dy, r.dz, __int_as_float(r.first));
            p.qout.s2[pos] = make_float4(r.hx, r.hy, r.hz, __int_as_float(r.id));
            p.qout.s3[pos] = make_float4(r.vx, r.vy, r.vz, __int_as_float(r.meta));
            p.qout.s4[pos] = make_double2(r.P, r.comp);
            p.qout.s5[pos] = make_double2(r.kdo, 0.0);
        }
    }
    flush_stats(p, bs);
}


// ---------------------------------------------------------------------------
// Primary-ray mask: one unit per (angle, node of its scene); every leaf child
// of the node marks the cells its box's projection (plus the plan's margin)
// touches.  Every leaf is the child of exactly one node, so the union over
// units is the silhouette of all leaf boxes of the scene at that angle.
// ---------------------------------------------------------------------------
constexpr int kMaskBlock = 256;
constexpr int kMaskMaxPerThread = 16;  // units of a thread, kMaskBlock apart, in large launches

// [min, max] of x . w over the box [lo, hi]
__device__ __forceinline__ void project_box(const double lo[3], const double hi[3], const double w[3], double &mn,
                                            double &mx)
{
    mn = 0.0;
    mx = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double a = lo[k] * w[k], b = hi[k] * w[k];
        mn += fmin(a, b);
        mx += fmax(a, b);
    }
}

// Ray indices [first, last] along one axis whose centres (c + (i + 0.5 - n / 2) ds)
// lie in [mn, mx] widened by `slack` spacings; false if none.
__device__ __forceinline__ bool ray_span(double mn, double mx, double c, double ds, int n, double slack, int &first,
                                         int &last)
{
    const double f0 = (mn - c) / ds + 0.5 * n - 0.5 - slack;
    const double f1 = (mx - c) / ds + 0.5 * n - 0.5 + slack;
    if (!(f1 >= 0.0) || !(f0 <= static_cast<double>(n - 1)) || !(f0 <= f1)) return false;
    first = static_cast<int>(ceil(fmax(f0, 0.0)));
    last = static_cast<int>(floor(fmin(f1, static_cast<double>(n - 1))));
    return first <= last;
}

__device__ void mask_box(const AnglePlan &pl, uint8_t *mask, const double lo[3], const double hi[3])
{
    double u0, u1, v0, v1;
    project_box(lo, hi, pl.u, u0, u1);
    project_box(lo, hi, pl.v, v0, v1);
    int i0, i1, j0, j1;
    if (!ray_span(u0, u1, pl.uc, pl.ds, pl.nu, pl.mslack, i0, i1)) return;
    if (!ray_span(v0, v1, pl.vc, pl.ds, pl.nv, pl.mslack, j0, j1)) return;
    for (int cj = j0 >> kMaskShift; cj <= (j1 >> kMaskShift); ++cj) {
        uint8_t *row = mask + pl.mask_base + static_cast<int64_t>(cj) * pl.mcu;
        for (int ci = i0 >> kMaskShift; ci <= (i1 >> kMaskShift); ++ci) row[ci] = 1;
    }
}

__global__ __launch_bounds__(kMaskBlock) void k_mask(const BNode *__restrict__ nodes,
                                                     const AnglePlan *__restrict__ plans, int n_angles,
                                                     int64_t n_units, int per_thread, uint8_t *__restrict__ mask)
{
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kMaskBlock * per_thread + threadIdx.x;
    if (first >= n_units) return;
    int a = 0, hi = n_angles;  // the angle of the first unit, then advanced
    while (hi - a > 1) {
        const int mid = (a + hi) >> 1;
        if (plans[mid].mwork_base <= first) a = mid;
        else hi = mid;
    }
    for (int k = 0; k < per_thread; ++k) {
        const int64_t g = first + static_cast<int64_t>(k) * kMaskBlock;
        if (g >= n_units) break;
        while (a + 1 < n_angles && plans[a + 1].mwork_base <= g) ++a;
        const AnglePlan &pl = plans[a];
        const BNode nd = nodes[pl.root + (g - pl.mwork_base)];
        if (nd.ch.x < 0) {
            const double lo[3] = {nd.a.x, nd.a.y, nd.a.z}, hi3[3] = {nd.a.w, nd.b.x, nd.b.y};
            mask_box(pl, mask, lo, hi3);
        }
        if (nd.ch.y < 0 && nd.ch.y != nd.ch.x) {
            const double lo[3] = {nd.b.z, nd.b.w, nd.c.x}, hi3[3] = {nd.c.y, nd.c.z, nd.c.w};
            mask_box(pl, mask, lo, hi3);
        }
    }
}

// ---------------------------------------------------------------------------
// Live tiles of a masked streaming launch: the tiles with a non-empty mask
// cell, in tile order.  The trace claims positions of this list, so a tile
// whose every ray the mask resolves is never claimed; its in-grid positions
// are counted here as masked queries, the count grid_ray makes ray by ray.
// Three launches: per-block counts, one block scanning them, the writes.
// ---------------------------------------------------------------------------
constexpr int kLiveBlock = 256;
constexpr int kLivePer = 4;  // consecutive tiles of a thread
constexpr int kLiveTiles = kLiveBlock * kLivePer;
constexpr int kLiveScanThreads = 1024;

// live flags of the thread's kLivePer tiles (bit j: tile first + j), the
// masked positions of the others in *masked
__device__ __forceinline__ uint32_t live_flags(const Params &p, int64_t first, uint32_t *masked)
{
    uint32_t f = 0, m = 0;
    for (int j = 0; j < kLivePer; ++j) {
        const int64_t t = first + j;
        if (t >= p.n_tiles) break;
        const int d = masked_tile(p, t, 0, p.n_angles - 1);
        if (d < 0) f |= 1u << j;
        else m += static_cast<uint32_t>(d);
    }
    *masked = m;
    return f;
}

// exclusive prefix of v over the block's threads (kLiveBlock), and the total
__device__ __forceinline__ uint32_t block_prefix(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kLiveBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;  // inclusive scan within the wave
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int k = 0; k < kLiveBlock / 64; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    *total = all;
    return before + x - v;
}

__global__ __launch_bounds__(kLiveBlock) void k_live_count(Params p, uint32_t *blk)
{
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kLiveTiles + static_cast<int64_t>(threadIdx.x) * kLivePer;
    uint32_t masked;
    const uint32_t f = live_flags(p, first, &masked);
    uint32_t n_live, n_masked;
    (void)block_prefix(static_cast<uint32_t>(__popc(f)), &n_live);
    __syncthreads();
    (void)block_prefix(masked, &n_masked);
    if (threadIdx.x == 0) {
        blk[blockIdx.x] = n_live;
        if (n_masked) {
            atomicAdd(p.stat + 0, static_cast<unsigned long long>(n_masked));
            atomicAdd(p.stat + kStatMasked, static_cast<unsigned long long>(n_masked));
        }
    }
}

// blk[0, nb) counts -> exclusive offsets, blk[nb] = the total
__global__ __launch_bounds__(kLiveScanThreads) void k_live_scan(uint32_t *blk, int64_t nb)
{
    __shared__ uint32_t part[kLiveScanThreads];
    const int t = threadIdx.x;
    const int64_t per = (nb + kLiveScanThreads - 1) / kLiveScanThreads;
    const int64_t lo = min(nb, per * t), hi = min(nb, lo + per);
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += blk[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < kLiveScanThreads; d <<= 1) {  // inclusive scan of part
        const uint32_t y = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t c = blk[i];
        blk[i] = run;
        run += c;
    }
    if (t == kLiveScanThreads - 1) blk[nb] = part[t];
}

__global__ __launch_bounds__(kLiveBlock) void k_live_write(Params p, const uint32_t *blk, int32_t *live)
{
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kLiveTiles + static_cast<int64_t>(threadIdx.x) * kLivePer;
    uint32_t masked, total;
    uint32_t f = live_flags(p, first, &masked);
    uint32_t o = blk[blockIdx.x] + block_prefix(static_cast<uint32_t>(__popc(f)), &total);
    for (int j = 0; f; ++j, f >>= 1)
        if (f & 1u) live[o++] = static_cast<int32_t>(first + j);
}

}  // namespace

int trace_block_threads() { return kBlock; }
int trace_stack_lds() { return kStackSpillLds; }
bool trace_needs_spill(const sbr_bvh *bvh, bool wide) { return stack_need(bvh, wide) > kStackLds; }
bool trace_walks_wide(const sbr_bvh *bvh, uint32_t flags, int schedule)
{
    return (flags & SBR_OPT_BVH4) && bvh->nodes4 != nullptr && bvh->scenes.empty() && schedule == kScheduleStream;
}

int trace_persistent_blocks(sbr_ctx *ctx, int blocks_per_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stream<0, false>, kBlock, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
    int blocks = ctx->prop.multiProcessorCount * per_cu;
    blocks = (blocks + 7) / 8 * 8;
    return blocks;
}

int check_tune(const sbr_tune &t)
{
    if (t.schedule != kScheduleStream && t.schedule != kScheduleWavefront)
        return fail(SBR_ERR_INVALID_ARG, "sbr_tune: schedule must be 0 or 1");
    if (t.tile_w != 4 && t.tile_w != 8 && t.tile_w != 16 && t.tile_w != 32 && t.tile_w != 64)
        return fail(SBR_ERR_INVALID_ARG, "sbr_tune: tile_w must be 4, 8, 16, 32 or 64");
    if (t.claim_tiles < 0 || t.claim_tiles > 64)
        return fail(SBR_ERR_INVALID_ARG, "sbr_tune: claim_tiles in [1, 64], or 0 (automatic)");
    if (t.refill_min < 1 || t.refill_min > 64) return fail(SBR_ERR_INVALID_ARG, "sbr_tune: refill_min in [1, 64]");
    if (t.blocks_per_cu < 0 || t.blocks_per_cu > 32)
        return fail(SBR_ERR_INVALID_ARG, "sbr_tune: blocks_per_cu in [0, 32]");
    if (t.chunk_log2 != 0 && (t.chunk_log2 < 16 || t.chunk_log2 > 30))
        return fail(SBR_ERR_INVALID_ARG, "sbr_tune: chunk_log2 must be 0 or in [16, 30]");
    return SBR_OK;
}

static Params make_params(const TraceArgs &a, int launch)
{
    Params p;
    p.nodes = a.bvh->nodes;
    p.nodes4 = trace_walks_wide(a.bvh, a.flags, a.schedule) ? a.bvh->nodes4 : nullptr;
    p.tris = a.bvh->tris;
    p.nrm = a.bvh->nrm_slot;
    p.eps = a.bvh->eps;
    {
        const SceneScale sc = scene_scale(a.bvh->bbox, a.bvh->diag);
        p.pbox = sc.pbox;
        p.obound = static_cast<float>(sc.obound);
        if (static_cast<double>(p.obound) > sc.obound) p.obound = std::nextafter(p.obound, 0.0f);
    }
    p.bmax = a.bmax;
    p.flags = a.flags;
    p.plans = a.plans;
    p.tile_base = a.tile_base;
    p.mask = a.mask;
    p.live = a.schedule == kScheduleStream ? a.live : nullptr;
    p.live_count = a.live_count;
    p.n_angles = a.n_angles;
    p.uo = a.rays ? a.rays->o : nullptr;
    p.ud = a.rays ? a.rays->d : nullptr;
    p.uh = a.rays ? a.rays->eH : nullptr;
    p.uv = a.rays ? a.rays->eV : nullptr;
    p.n_rays = a.n_rays;
    p.hits = a.hits ? *a.hits : sbr_hits{};
    p.kx = a.k_hat[0];
    p.ky = a.k_hat[1];
    p.kz = a.k_hat[2];
    p.qin = a.q_in;
    p.qout = a.q_out;
    p.qin_cnt = a.ctrs.q_cnt + (launch - 1) * kLineU32;
    p.qout_cnt = a.ctrs.q_cnt + launch * kLineU32;
    p.rec = a.rec;
    p.n_tiles = a.n_tiles;
    p.ctr = a.ctrs.claim + static_cast<size_t>(launch) * kClaimRanges * kLineU32;
    p.stat = a.ctrs.stat;
    p.spill = a.spill;
    p.bounce = launch;
    p.user_sink = a.hits != nullptr;
    p.tile_shift = a.tile_shift;
    p.claim_tiles = a.claim_tiles;
    p.refill_min = a.refill_min;
    p.packet = (a.flags & SBR_OPT_PACKET) && !(a.flags & SBR_OPT_FP64_TRAVERSE) && p.nodes4 == nullptr &&
               stack_need(a.bvh, false) <= kPacketStack;
    return p;
}

template <bool SPILL>
static void launch_trace_t(hipStream_t s, const TraceArgs &a, const Params &p, int bounce)
{
    const bool user = a.hits != nullptr;
    if (a.schedule == kScheduleStream) {
        const bool wide = p.nodes4 != nullptr;
        if (a.flags & SBR_OPT_FP64_TRAVERSE) {
            if (wide) {
                if (user) k_stream<1, SPILL, double, 4><<<a.blocks, kBlock, 0, s>>>(p);
                else k_stream<0, SPILL, double, 4><<<a.blocks, kBlock, 0, s>>>(p);
            } else {
                if (user) k_stream<1, SPILL, double><<<a.blocks, kBlock, 0, s>>>(p);
                else k_stream<0, SPILL, double><<<a.blocks, kBlock, 0, s>>>(p);
            }
        } else if (wide) {
            if (user) k_stream<1, SPILL, float, 4><<<a.blocks, kBlock, 0, s>>>(p);
            else k_stream<0, SPILL, float, 4><<<a.blocks, kBlock, 0, s>>>(p);
        } else {
            if (user) k_stream<1, SPILL><<<a.blocks, kBlock, 0, s>>>(p);
            else k_stream<0, SPILL><<<a.blocks, kBlock, 0, s>>>(p);
        }
    } else if (bounce == 1) {
        if (user) k_wave<1, SPILL><<<a.blocks, kBlock, 0, s>>>(p);
        else k_wave<0, SPILL><<<a.blocks, kBlock, 0, s>>>(p);
    } else {
        k_wave<2, SPILL><<<a.blocks, kBlock, 0, s>>>(p);
    }
}

int launch_mask(hipStream_t s, const BNode *nodes, const AnglePlan *plans, int n_angles, int64_t n_units,
                uint8_t *mask, int64_t mask_bytes)
{
    if (mask_bytes % 4 != 0 || n_angles < 1) return fail(SBR_ERR_INVALID_ARG, "launch_mask: bad layout");
    int rc;
    if ((rc = launch_zero_u32(s, reinterpret_cast<uint32_t *>(mask), mask_bytes / 4))) return rc;
    // at least ~4,096 workgroups before a thread takes several units
    const int per = static_cast<int>(
        std::min<int64_t>(kMaskMaxPerThread, std::max<int64_t>(1, n_units / (int64_t(kMaskBlock) * 4096))));
    const int64_t per_block = static_cast<int64_t>(kMaskBlock) * per;
    const int64_t blocks = (n_units + per_block - 1) / per_block;
    if (blocks > 0)
        k_mask<<<static_cast<unsigned>(blocks), kMaskBlock, 0, s>>>(nodes, plans, n_angles, n_units, per, mask);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int64_t live_blocks(int64_t n_tiles) { return (n_tiles + kLiveTiles - 1) / kLiveTiles; }

int launch_live(hipStream_t s, const TraceArgs &a, int32_t *live, uint32_t *blk)
{
    if (!a.mask || a.n_angles < 1 || a.n_tiles < 1) return fail(SBR_ERR_INVALID_ARG, "launch_live: bad launch");
    if (a.n_tiles > INT32_MAX) return fail(SBR_ERR_OVERFLOW, "launch_live: too many tiles in one launch");
    Params p{};
    p.plans = a.plans;
    p.tile_base = a.tile_base;
    p.mask = a.mask;
    p.n_angles = a.n_angles;
    p.n_tiles = a.n_tiles;
    p.tile_shift = a.tile_shift;
    p.stat = a.ctrs.stat;
    const int64_t nb = live_blocks(a.n_tiles);
    k_live_count<<<static_cast<unsigned>(nb), kLiveBlock, 0, s>>>(p, blk);
    k_live_scan<<<1, kLiveScanThreads, 0, s>>>(blk, nb);
    k_live_write<<<static_cast<unsigned>(nb), kLiveBlock, 0, s>>>(p, blk, live);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

// ---------------------------------------------------------------------------
// Static scratch of sbr_trace_noalloc (for callers that cannot allocate
// device memory): the counter block of one streaming trace, laid out as
//   [0, kStatBytes)               stat (u64 counters)
//   2 lines                       q_cnt of launches 0 and 1 (not read by the
//                                 streaming schedule, but addressed)
//   2 x kClaimRanges lines        claim counters of launches 0 and 1
// Every device holds its own copy of the array at its own address.  In host
// code the array's name is not a device address: the address of each
// device's copy is looked up once, with that device current, and only that
// pointer is handed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kNoallocQcntOff = kStatBytes;
constexpr size_t kNoallocClaimOff = kNoallocQcntOff + 2 * 4 * kLineU32;
constexpr size_t kNoallocUsed = kNoallocClaimOff + 2 * size_t(kClaimRanges) * 4 * kLineU32;
static_assert(kNoallocUsed <= kNoallocScratchBytes, "the no-alloc counter layout fits its scratch");

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(SBR_ERR_UNSUPPORTED, "no-alloc scratch: device index beyond " + std::to_string(kMaxDevices));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return SBR_OK;
    int cur = -1;
    SBR_HIP(hipGetDevice(&cur));
    if (cur != device) return fail(SBR_ERR_INVALID_ARG, "no-alloc scratch: set up with another device current");
    void *ptr = nullptr;
    SBR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SBR_ERR_HIP, "no-alloc scratch: hipGetSymbolAddress gave no address");
    g_scratch_ptr[device] = ptr;
    return SBR_OK;
}

int noalloc_counters(int device, CounterPtrs &c, void **base, size_t *bytes)
{
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (device >= 0 && device < kMaxDevices) ptr = g_scratch_ptr[device];
    }
    if (!ptr) return fail(SBR_ERR_INVALID_ARG, "no-alloc scratch of this device was not set up (sbr_create)");
    char *b = static_cast<char *>(ptr);
    c.stat = reinterpret_cast<unsigned long long *>(b);
    c.q_cnt = reinterpret_cast<uint32_t *>(b + kNoallocQcntOff);
    c.claim = reinterpret_cast<uint32_t *>(b + kNoallocClaimOff);
    *base = ptr;
    *bytes = kNoallocUsed;
    return SBR_OK;
}

int launch_trace(hipStream_t s, const TraceArgs &a, int bounce)
{
    const Params p = make_params(a, bounce);
    // the stack holds at most one entry per level of the current path (three for a BVH4)
    if (trace_needs_spill(a.bvh, p.nodes4 != nullptr)) launch_trace_t<true>(s, a, p, bounce);
    else launch_trace_t<false>(s, a, p, bounce);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

}  // namespace sbr
