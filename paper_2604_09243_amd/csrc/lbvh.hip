// GPU BVH construction: linear BVH and PLOC, on one shared Morton sort.
//
// The paper builds a median / binned-SAH BVH recursively on the host
// (Sec. 4, Algorithm 1).  Here the tree is built on the device in
// data-parallel passes:
//   1. 63-bit Morton code of each triangle centroid (21 bits per axis);
//   2. stable LSD radix sort of (code, triangle) in eight 8-bit passes, each
//      pass a per-tile LDS histogram, one scan of all tile histograms, and an
//      LDS-ranked scatter (wave ballots give the rank among equal digits).
// LBVH (build_lbvh):
//   3. the radix-tree hierarchy over the sorted codes (one thread per
//      internal node, longest-common-prefix split search; equal codes are
//      separated by their sorted index);
//   4. bottom-up refit of padded boxes: one thread per leaf climbs towards
//      the root and stops at the first parent whose other child is not done
//      yet (per-node arrival counter);
//   5. relayout into preorder, with both child boxes stored in the parent.
//   Subtrees of at most leaf_max triangles are collapsed into leaves (their
//   triangles are contiguous in sorted order), the leaf threshold of the
//   paper's build.
// PLOC (build_ploc): bottom-up agglomerative clustering along the sorted
// order (parallel locally-ordered clustering): every cluster finds the
// neighbour within kPlocRadius positions whose merged box has the smallest
// surface area, mutual nearest neighbours merge, the survivors are compacted
// in order, until one cluster is left.  A merge decides at once, from the
// surface-area cost of its two subtrees, whether a subtree of at most
// leaf_max triangles is cheaper as a leaf.  Large cluster counts iterate as
// four launches per step; at most kPlocSmall clusters finish inside one
// workgroup in LDS.  A walk to the root then gives every kept node its
// preorder index and every triangle its slot in leaf order.  The tree has
// the surface-area quality of the host SAH build at GPU build speed.
// Boxes are padded so the traversal's box test never culls a triangle the
// float32 intersection test would accept.
#include <algorithm>
#include <cmath>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

constexpr int kSortThreads = 256;
constexpr int kLeafMaxLimit = 4;  // the leaf code keeps 2 count bits
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

__device__ inline uint64_t spread21(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ void k_morton(const float *__restrict__ v0, const float *__restrict__ e1, const float *__restrict__ e2,
                         int n, float lox, float loy, float loz, float sx, float sy, float sz,
                         uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float third = 1.0f / 3.0f;
    float c[3];
    for (int a = 0; a < 3; ++a) c[a] = v0[3 * i + a] + (e1[3 * i + a] + e2[3 * i + a]) * third;
    const float lo[3] = {lox, loy, loz}, sc[3] = {sx, sy, sz};
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        float f = (c[a] - lo[a]) * sc[a];
        f = fminf(fmaxf(f, 0.0f), 2097151.0f);
        q[a] = static_cast<uint32_t>(f);
    }
    keys[i] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
    vals[i] = static_cast<uint32_t>(i);
}

__global__ __launch_bounds__(kSortThreads) void k_hist(const uint64_t *__restrict__ keys, int n, int shift,
                                                       uint32_t *__restrict__ hist, int nblocks)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = base + k * kSortThreads + tid;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[static_cast<int64_t>(tid) * nblocks + blockIdx.x] = h[tid];
}

// Exclusive scan of m values in place, one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(uint32_t *__restrict__ data, int m)
{
    __shared__ uint32_t s[1024];
    const int tid = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int b = tid * per, e = min(b + per, m);
    uint32_t sum = 0;
    for (int i = b; i < e; ++i) sum += data[i];
    s[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = tid >= off ? s[tid - off] : 0u;
        __syncthreads();
        s[tid] += v;
        __syncthreads();
    }
    uint32_t run = s[tid] - sum;
    for (int i = b; i < e; ++i) {
        const uint32_t x = data[i];
        data[i] = run;
        run += x;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_scatter(const uint64_t *__restrict__ kin,
                                                          const uint32_t *__restrict__ vin,
                                                          uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                          int n, int shift, const uint32_t *__restrict__ hist,
                                                          int nblocks)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    base[tid] = hist[static_cast<int64_t>(tid) * nblocks + blockIdx.x];
    run[tid] = 0;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = static_cast<int64_t>(blockIdx.x) * kSortTile + k * kSortThreads + tid;
        const bool valid = idx < n;
        const uint64_t key = valid ? kin[idx] : 0ull;
        const uint32_t val = valid ? vin[idx] : 0u;
        const uint32_t digit = valid ? static_cast<uint32_t>((key >> shift) & 255u) : 0u;
        for (int d = tid; d < 4 * 256; d += kSortThreads) (&wcnt[0][0])[d] = 0;
        __syncthreads();
        uint64_t eq = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const uint64_t m = __ballot(bit);
            eq &= bit ? m : ~m;
        }
        if (!valid) eq = 0;
        const uint32_t rank = __popcll(eq & lt);
        if (valid && rank == 0) wcnt[w][digit] = __popcll(eq);
        __syncthreads();
        {
            const int d = tid;
            const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
            const uint32_t r = run[d];
            wcnt[0][d] = r;
            wcnt[1][d] = r + c0;
            wcnt[2][d] = r + c0 + c1;
            wcnt[3][d] = r + c0 + c1 + c2;
            run[d] = r + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = base[digit] + wcnt[w][digit] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

// At most kSmallSort keys: one workgroup sorts (code, index) pairs by a
// bitonic network in LDS.  Ordering the pairs lexicographically gives the
// same order as the stable radix sort (indices are unique); padding pairs
// compare above every real one.
constexpr int kSmallSort = 2048;

__global__ __launch_bounds__(kSmallSort / 2) void k_sort_small(const uint64_t *__restrict__ kin,
                                                               const uint32_t *__restrict__ vin, int n,
                                                               uint64_t *__restrict__ kout,
                                                               uint32_t *__restrict__ vout)
{
    __shared__ uint64_t sk[kSmallSort];
    __shared__ uint32_t sv[kSmallSort];
    const int tid = threadIdx.x;
    for (int k = tid; k < kSmallSort; k += kSmallSort / 2) {
        sk[k] = k < n ? kin[k] : ~0ull;
        sv[k] = k < n ? vin[k] : 0xffffffffu;
    }
    __syncthreads();
    for (int size = 2; size <= kSmallSort; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int i = 2 * stride * (tid / stride) + (tid % stride), j = i + stride;
            const uint64_t ki = sk[i], kj = sk[j];
            const uint32_t vi = sv[i], vj = sv[j];
            const bool gt = ki > kj || (ki == kj && vi > vj);
            if (gt == ((i & size) == 0)) {
                sk[i] = kj;
                sk[j] = ki;
                sv[i] = vj;
                sv[j] = vi;
            }
            __syncthreads();
        }
    }
    for (int k = tid; k < n; k += kSmallSort / 2) {
        kout[k] = sk[k];
        vout[k] = sv[k];
    }
}

__device__ inline int lcp(const uint64_t *__restrict__ k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz(static_cast<uint32_t>(i ^ j));
    return __clzll(a ^ b);
}

// One thread per internal node i in [0, n-2]; children encoded as
// internal >= 0, leaf = ~index.
__global__ void k_karras(const uint64_t *__restrict__ keys, int n, int *__restrict__ left, int *__restrict__ right,
                         int *__restrict__ parent_int, int *__restrict__ parent_leaf, int *__restrict__ range_first,
                         int *__restrict__ range_last, uint8_t *__restrict__ is_left)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (lcp(keys, n, i, i + 1) - lcp(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = lcp(keys, n, i, i - d);
    int lmax = 2;
    while (lcp(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (lcp(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = lcp(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (lcp(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    int lc, rc;
    if (lo == gamma) {
        lc = ~gamma;
        parent_leaf[gamma] = i;
    } else {
        lc = gamma;
        parent_int[gamma] = i;
        is_left[gamma] = 1;
    }
    if (hi == gamma + 1) {
        rc = ~(gamma + 1);
        parent_leaf[gamma + 1] = i;
    } else {
        rc = gamma + 1;
        parent_int[gamma + 1] = i;
        is_left[gamma + 1] = 0;
    }
    left[i] = lc;
    right[i] = rc;
    range_first[i] = lo;
    range_last[i] = hi;
    if (i == 0) parent_int[0] = -1;
}

// Box of the triangle at sorted position j: the hit rule's box (widened by
// P) widened by the guard G (SceneScale).
__device__ inline void leaf_box(const uint32_t *__restrict__ order, const float *__restrict__ v0,
                                const float *__restrict__ e1, const float *__restrict__ e2, float P, float G, int j,
                                float *lo, float *hi)
{
    const int li = static_cast<int>(order[j]);
    const float *a = v0 + 3 * li, *b = e1 + 3 * li, *c = e2 + 3 * li;
    for (int k = 0; k < 3; ++k) {
        float l, h;
        spec_box_axis(a[k], b[k], c[k], P, l, h);
        lo[k] = l - G;
        hi[k] = h + G;
    }
}

// Leaf boxes in sorted order: lbox[6 j ..] = lo xyz, hi xyz.
__global__ void k_leaf_boxes(int n, const uint32_t *__restrict__ order, const float *__restrict__ v0,
                             const float *__restrict__ e1, const float *__restrict__ e2, float P, float G,
                             float *__restrict__ lbox)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    leaf_box(order, v0, e1, e2, P, G, j, lbox + 6 * j, lbox + 6 * j + 3);
}

// Triangles and their normals at their leaf slots: the triangle at sorted
// position j goes to slot slot_of[j] (slot j when slot_of is null).
__global__ void k_place(int n, const uint32_t *__restrict__ order, const int *__restrict__ slot_of,
                        const float *__restrict__ v0, const float *__restrict__ e1, const float *__restrict__ e2,
                        const float *__restrict__ nrm, const int32_t *__restrict__ ids, BTri *__restrict__ tris,
                        float4 *__restrict__ nrm_slot)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int li = static_cast<int>(order[j]);
    const int slot = slot_of ? slot_of[j] : j;
    if (slot < 0 || slot >= n) return;  // the builder's checks report a bad permutation
    const float *a = v0 + 3 * li, *b = e1 + 3 * li, *c = e2 + 3 * li;
    BTri t;
    t.p0 = make_float4(a[0], a[1], a[2], __int_as_float(ids[li]));
    t.p1 = make_float4(b[0], b[1], b[2], 0.0f);
    t.p2 = make_float4(c[0], c[1], c[2], 0.0f);
    tris[slot] = t;
    nrm_slot[slot] = make_float4(nrm[3 * li], nrm[3 * li + 1], nrm[3 * li + 2], 0.0f);
}

__device__ inline float aload(const float *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_refit(int n, const int *__restrict__ left, const int *__restrict__ right,
                        const int *__restrict__ parent_int, const int *__restrict__ parent_leaf,
                        const float *lbox, float *nbox, int *arrive)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int node = parent_leaf[j];
    while (node >= 0) {
        __threadfence();
        if (atomicAdd(&arrive[node], 1) == 0) return;  // the sibling subtree is not finished yet
        __threadfence();
        const int c[2] = {left[node], right[node]};
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int s = 0; s < 2; ++s) {
            const float *b = c[s] < 0 ? lbox + 6 * (~c[s]) : nbox + 6 * c[s];
            for (int k = 0; k < 3; ++k) {
                lo[k] = fminf(lo[k], aload(b + k));
                hi[k] = fmaxf(hi[k], aload(b + 3 + k));
            }
        }
        for (int k = 0; k < 3; ++k) {
            __hip_atomic_store(nbox + 6 * node + k, lo[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(nbox + 6 * node + 3 + k, hi[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        node = parent_int[node];
    }
}

// Preorder position of internal node i: the first leaf of its range plus the
// number of "left child" edges on its path from the root.
__global__ void k_preorder(int n_int, const int *__restrict__ parent_int, const uint8_t *__restrict__ is_left,
                           const int *__restrict__ range_first, int *__restrict__ pre, int *__restrict__ depth)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    int cnt = 0, dep = 0, node = i;
    while (parent_int[node] >= 0) {
        cnt += is_left[node];
        ++dep;
        node = parent_int[node];
    }
    pre[i] = range_first[i] + cnt;
    atomicMax(depth, dep + 1);
}

// Internal nodes whose range holds more than leaf_max triangles are kept;
// flag them at their full preorder position so a scan numbers the kept
// nodes in preorder.
__global__ void k_mark_kept(int n_int, const int *__restrict__ pre, const int *__restrict__ range_first,
                            const int *__restrict__ range_last, int leaf_max, uint32_t *__restrict__ flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    flag[pre[i]] = (range_last[i] - range_first[i] + 1 > leaf_max) ? 1u : 0u;
}

__device__ inline int leaf_ref(int first, int count) { return ~((first << 3) | (count - 1)); }

__global__ void k_relayout(int n_int, const int *__restrict__ left, const int *__restrict__ right,
                           const int *__restrict__ pre, const uint32_t *__restrict__ newidx,
                           const int *__restrict__ range_first, const int *__restrict__ range_last, int leaf_max,
                           const float *__restrict__ lbox, const float *__restrict__ nbox, BNode *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    if (range_last[i] - range_first[i] + 1 <= leaf_max) return;  // inside a collapsed leaf
    const int c[2] = {left[i], right[i]};
    float bx[2][6];
    int ref[2];
    for (int s = 0; s < 2; ++s) {
        const float *b = c[s] < 0 ? lbox + 6 * (~c[s]) : nbox + 6 * c[s];
        for (int k = 0; k < 6; ++k) bx[s][k] = b[k];
        if (c[s] < 0) {
            ref[s] = leaf_ref(~c[s], 1);
        } else {
            const int cnt = range_last[c[s]] - range_first[c[s]] + 1;
            ref[s] = cnt <= leaf_max ? leaf_ref(range_first[c[s]], cnt) : static_cast<int>(newidx[pre[c[s]]]);
        }
    }
    BNode nd;
    nd.a = make_float4(bx[0][0], bx[0][1], bx[0][2], bx[0][3]);
    nd.b = make_float4(bx[0][4], bx[0][5], bx[1][0], bx[1][1]);
    nd.c = make_float4(bx[1][2], bx[1][3], bx[1][4], bx[1][5]);
    nd.ch = make_int4(ref[0], ref[1], 0, 0);
    out[newidx[pre[i]]] = nd;
}

// Tree of at most leaf_max triangles: one node whose two children are the
// same leaf (tested twice, with the same result).
__global__ void k_single(int n, const float *__restrict__ lbox, BNode *__restrict__ out)
{
    float b[6];
    for (int k = 0; k < 3; ++k) {
        b[k] = INFINITY;
        b[3 + k] = -INFINITY;
    }
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < 3; ++k) {
            b[k] = fminf(b[k], lbox[6 * j + k]);
            b[3 + k] = fmaxf(b[3 + k], lbox[6 * j + 3 + k]);
        }
    BNode nd;
    nd.a = make_float4(b[0], b[1], b[2], b[3]);
    nd.b = make_float4(b[4], b[5], b[0], b[1]);
    nd.c = make_float4(b[2], b[3], b[4], b[5]);
    nd.ch = make_int4(leaf_ref(0, n), leaf_ref(0, n), 0, 0);
    out[0] = nd;
}

// ------------------------------------------------------------------ PLOC
// Clusters are (lo.xyz, reference) and (hi.xyz, subtree cost) float4 pairs;
// a reference is ~j for the triangle at sorted position j and p for
// internal node p.  Internal nodes are numbered in creation order, so a
// parent's index is larger than its children's and the root is n - 2.

#ifndef SBR_PLOC_RADIUS
#define SBR_PLOC_RADIUS 16
#endif
constexpr int kPlocRadius = SBR_PLOC_RADIUS;  // neighbours searched on each side in the sorted order
constexpr int kPlocTile = 256;    // clusters per workgroup of the iterated steps
constexpr int kPlocSmall = 2048;  // clusters finished inside one workgroup
constexpr int kPlocSmallThreads = 1024;
constexpr int kPlocPer = kPlocSmall / kPlocSmallThreads;
constexpr int kPlocMaxSteps = 1 << 16;
// A node visit (two box tests) in triangle tests, the host SAH build's
// measured constant (0.5 → 1.5: batch 3.16 → 2.90 s, aircraft 8.84 → 8.34 ms).
constexpr float kPlocNodeCost = 1.5f;

struct PlocState {
    int m;          // live clusters
    int node_base;  // internal nodes created so far
    int pad[2];
};

struct PlocNodes {
    float4 *lo;  // box lo, w = surface-area cost of the subtree
    float4 *hi;  // box hi, w = triangle count (int bits)
    int2 *ch;    // children (the cluster references)
    int *kept;   // internal nodes of the layout at and below this node; 0 = the subtree is one leaf
    int *pint;   // parent of an internal node: (p << 1) | (1 for the right child); -1 at the root
    int *pleaf;  // parent of the triangle at a sorted position, same code
};

__device__ inline int aload_i(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Half the surface area of a box.
__device__ inline float half_area(float lx, float ly, float lz, float hx, float hy, float hz)
{
    const float dx = hx - lx, dy = hy - ly, dz = hz - lz;
    return dx * dy + dy * dz + dz * dx;
}

// Half the surface area of the union of two boxes (symmetric in the two).
__device__ inline float merged_area(const float4 &la, const float4 &ha, const float4 &lb, const float4 &hb)
{
    return half_area(fminf(la.x, lb.x), fminf(la.y, lb.y), fminf(la.z, lb.z), fmaxf(ha.x, hb.x),
                     fmaxf(ha.y, hb.y), fmaxf(ha.z, hb.z));
}

// Nearest neighbour of cluster i among positions [i - R, i + R] of [0, m):
// the smallest merged area, ties to the smallest position.  That is a total
// order on pairs, so the best pair of a step is mutual and every step merges.
// lo/hi hold positions [off, ...).
__device__ inline int ploc_nn(int i, int m, const float4 *lo, const float4 *hi, int off)
{
    const float4 li = lo[i - off], hi_i = hi[i - off];
    float best = 0.0f;
    int bj = -1;
    const int j0 = max(0, i - kPlocRadius), j1 = min(m - 1, i + kPlocRadius);
    for (int j = j0; j <= j1; ++j) {
        if (j == i) continue;
        const float a = merged_area(li, hi_i, lo[j - off], hi[j - off]);
        if (bj < 0 || a < best) {
            best = a;
            bj = j;
        }
    }
    return bj;
}

// Cluster i survives the step (keep) and merges with its neighbour (merge,
// the lower position of a mutual pair).
template <class I>
__device__ inline void ploc_flags(const I *nn, int i, int m, bool &keep, bool &merge)
{
    keep = merge = false;
    if (i >= m) return;
    const int j = nn[i];
    if (j < 0) {
        keep = true;
        return;
    }
    const bool mutual = static_cast<int>(nn[j]) == i;
    merge = mutual && i < j;
    keep = !(mutual && i > j);
}

// (triangle count, kept nodes) of the subtree behind a cluster, for a
// cluster held in global memory (nodes written by earlier launches).
__device__ inline int2 cluster_stats(const float4 &lo, const PlocNodes &nd)
{
    const int c = __float_as_int(lo.w);
    if (c < 0) return make_int2(1, 0);
    return make_int2(__float_as_int(aload(&nd.hi[c].w)), aload_i(&nd.kept[c]));
}

// Node p from the clusters (la, ha, sa) and (lb, hb, sb); the merged
// cluster goes to (olo, ohi) and its stats are returned.  A cluster's hi.w
// is its subtree cost, in units of one triangle test per unit of half area
// with a node visit counted as kPlocNodeCost triangle tests (the host SAH
// build's constant): a subtree of at most leaf_max triangles becomes one
// leaf when that costs no more than the node and its two subtrees.
__device__ inline int2 ploc_merge(int p, const float4 &la, const float4 &ha, int2 sa, const float4 &lb,
                                  const float4 &hb, int2 sb, const PlocNodes &nd, int leaf_max, float4 &olo,
                                  float4 &ohi)
{
    const float lx = fminf(la.x, lb.x), ly = fminf(la.y, lb.y), lz = fminf(la.z, lb.z);
    const float hx = fmaxf(ha.x, hb.x), hy = fmaxf(ha.y, hb.y), hz = fmaxf(ha.z, hb.z);
    const float A = half_area(lx, ly, lz, hx, hy, hz);
    const int cnt = sa.x + sb.x;
    const float c_node = kPlocNodeCost * A + ha.w + hb.w;
    const float c_leaf = A * static_cast<float>(cnt);
    const bool leaf = cnt <= leaf_max && c_leaf <= c_node;
    const float cost = leaf ? c_leaf : c_node;
    const int kept = leaf ? 0 : 1 + sa.y + sb.y;
    const int a = __float_as_int(la.w), b = __float_as_int(lb.w);
    nd.lo[p] = make_float4(lx, ly, lz, cost);
    nd.hi[p] = make_float4(hx, hy, hz, __int_as_float(cnt));
    nd.ch[p] = make_int2(a, b);
    nd.kept[p] = kept;
    if (a < 0)
        nd.pleaf[~a] = p << 1;
    else
        nd.pint[a] = p << 1;
    if (b < 0)
        nd.pleaf[~b] = (p << 1) | 1;
    else
        nd.pint[b] = (p << 1) | 1;
    olo = make_float4(lx, ly, lz, __int_as_float(p));
    ohi = make_float4(hx, hy, hz, cost);
    return make_int2(cnt, kept);
}

// One cluster per triangle, in sorted order.
__global__ void k_ploc_init(int n, const float *__restrict__ lbox, float4 *__restrict__ lo, float4 *__restrict__ hi,
                            PlocState *__restrict__ st)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {
        st->m = n;
        st->node_base = 0;
    }
    if (j >= n) return;
    const float *b = lbox + 6 * j;
    lo[j] = make_float4(b[0], b[1], b[2], __int_as_float(~j));
    hi[j] = make_float4(b[3], b[4], b[5], half_area(b[0], b[1], b[2], b[3], b[4], b[5]));
}

// Step, part 1: nearest neighbours (cluster boxes of the tile and its halo in LDS).
__global__ __launch_bounds__(kPlocTile) void k_ploc_nn(const PlocState *__restrict__ st,
                                                       const float4 *__restrict__ lo, const float4 *__restrict__ hi,
                                                       int *__restrict__ nn)
{
    __shared__ float4 slo[kPlocTile + 2 * kPlocRadius], shi[kPlocTile + 2 * kPlocRadius];
    const int m = st->m;
    const int t0 = blockIdx.x * kPlocTile;
    if (t0 >= m) return;
    const int off = t0 - kPlocRadius;
    for (int k = threadIdx.x; k < kPlocTile + 2 * kPlocRadius; k += kPlocTile) {
        const int g = off + k;
        if (g >= 0 && g < m) {
            slo[k] = lo[g];
            shi[k] = hi[g];
        }
    }
    __syncthreads();
    const int i = t0 + threadIdx.x;
    if (i < m) nn[i] = m > 1 ? ploc_nn(i, m, slo, shi, off) : -1;
}

// Step, part 2: per-tile counts of surviving clusters (x) and merges (y).
__global__ __launch_bounds__(kPlocTile) void k_ploc_count(const PlocState *__restrict__ st,
                                                          const int *__restrict__ nn, uint2 *__restrict__ tc)
{
    __shared__ uint32_t wk[kPlocTile / 64], wm[kPlocTile / 64];
    const int m = st->m;
    const int t0 = blockIdx.x * kPlocTile;
    if (t0 >= m) return;
    bool keep, merge;
    ploc_flags(nn, t0 + static_cast<int>(threadIdx.x), m, keep, merge);
    const uint64_t bk = __ballot(keep), bm = __ballot(merge);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        wk[w] = __popcll(bk);
        wm[w] = __popcll(bm);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int v = 0; v < kPlocTile / 64; ++v) {
            a += wk[v];
            b += wm[v];
        }
        tc[blockIdx.x] = make_uint2(a, b);
    }
}

// Step, part 3: exclusive scan of the tile counts (one workgroup); the next
// step's cluster count and node base go to nxt.
__global__ __launch_bounds__(1024) void k_ploc_scan(const PlocState *__restrict__ st, PlocState *__restrict__ nxt,
                                                    uint2 *__restrict__ tc)
{
    __shared__ uint32_t sa[1024], sb[1024];
    const int tid = threadIdx.x;
    const int m = st->m;
    const int nt = (m + kPlocTile - 1) / kPlocTile;
    const int per = (nt + 1023) / 1024;
    const int b = tid * per, e = min(b + per, nt);
    uint32_t ka = 0, kb = 0;
    for (int i = b; i < e; ++i) {
        ka += tc[i].x;
        kb += tc[i].y;
    }
    sa[tid] = ka;
    sb[tid] = kb;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t va = tid >= off ? sa[tid - off] : 0u, vb = tid >= off ? sb[tid - off] : 0u;
        __syncthreads();
        sa[tid] += va;
        sb[tid] += vb;
        __syncthreads();
    }
    uint32_t ra = sa[tid] - ka, rb = sb[tid] - kb;
    for (int i = b; i < e; ++i) {
        const uint2 x = tc[i];
        tc[i] = make_uint2(ra, rb);
        ra += x.x;
        rb += x.y;
    }
    if (tid == 1023) {
        nxt->m = static_cast<int>(sa[1023]);
        nxt->node_base = st->node_base + static_cast<int>(sb[1023]);
    }
}

// Step, part 4: merges write their nodes, survivors are compacted in order.
__global__ __launch_bounds__(kPlocTile) void k_ploc_apply(const PlocState *__restrict__ st,
                                                          const int *__restrict__ nn, const uint2 *__restrict__ tc,
                                                          const float4 *__restrict__ lo, const float4 *__restrict__ hi,
                                                          float4 *__restrict__ olo, float4 *__restrict__ ohi,
                                                          PlocNodes nd, int leaf_max, int n_int,
                                                          int *__restrict__ err)
{
    __shared__ uint32_t wk[kPlocTile / 64], wm[kPlocTile / 64];
    const int m = st->m, node_base = st->node_base;
    const int t0 = blockIdx.x * kPlocTile;
    if (t0 >= m) return;
    const int i = t0 + static_cast<int>(threadIdx.x);
    bool keep, merge;
    ploc_flags(nn, i, m, keep, merge);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint64_t bk = __ballot(keep), bm = __ballot(merge);
    if (lane == 0) {
        wk[w] = __popcll(bk);
        wm[w] = __popcll(bm);
    }
    __syncthreads();
    uint32_t ok = tc[blockIdx.x].x, om = tc[blockIdx.x].y;
    for (int v = 0; v < w; ++v) {
        ok += wk[v];
        om += wm[v];
    }
    const int kpos = static_cast<int>(ok + __popcll(bk & lt)), mpos = static_cast<int>(om + __popcll(bm & lt));
    if (merge) {
        const int j = nn[i];
        if (node_base + mpos < n_int) {
            const float4 li = lo[i], lj = lo[j];
            ploc_merge(node_base + mpos, li, hi[i], cluster_stats(li, nd), lj, hi[j], cluster_stats(lj, nd), nd,
                       leaf_max, olo[kpos], ohi[kpos]);
        } else
            *err = 4;
    } else if (keep) {
        olo[kpos] = lo[i];
        ohi[kpos] = hi[i];
    }
}

// The last kPlocSmall clusters: every step inside one workgroup.  Clusters
// and their (count, kept) stats live in LDS; a step gathers each thread's
// clusters and merge partners into registers, then writes the compacted
// array in place, so no global memory is read inside the loop (nodes are
// only written).  err: 1 = too many clusters, 2 = no single root.
__global__ __launch_bounds__(kPlocSmallThreads) void k_ploc_small(const PlocState *__restrict__ st,
                                                                  const float4 *__restrict__ lo,
                                                                  const float4 *__restrict__ hi, PlocNodes nd,
                                                                  int leaf_max, int n_int, int *__restrict__ err)
{
    __shared__ float4 slo[kPlocSmall], shi[kPlocSmall];
    __shared__ int2 sst[kPlocSmall];
    __shared__ int16_t snn[kPlocSmall];
    __shared__ uint32_t wsum[kPlocSmallThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int m = st->m, node_base = st->node_base;
    if (m > kPlocSmall || m < 1) {
        if (tid == 0) *err = 1;
        return;
    }
    for (int k = tid; k < m; k += kPlocSmallThreads) {
        const float4 l = lo[k];
        slo[k] = l;
        shi[k] = hi[k];
        const int c = __float_as_int(l.w);
        sst[k] = c < 0 ? make_int2(1, 0) : make_int2(__float_as_int(nd.hi[c].w), nd.kept[c]);
    }
    __syncthreads();
    const int i0 = tid * kPlocPer;
    for (int step = 0; m > 1 && step < kPlocSmall; ++step) {
        // neighbour search with consecutive lanes on consecutive clusters
        // (conflict-free LDS reads); the scan below owns contiguous pairs
        for (int q = 0; q < kPlocPer; ++q) {
            const int i = tid + q * kPlocSmallThreads;
            if (i < m) snn[i] = static_cast<int16_t>(ploc_nn(i, m, slo, shi, 0));
        }
        __syncthreads();
        bool kf[kPlocPer], mf[kPlocPer];
        uint32_t c = 0;
        for (int q = 0; q < kPlocPer; ++q) {
            ploc_flags(snn, i0 + q, m, kf[q], mf[q]);
            c += (kf[q] ? 1u : 0u) + (mf[q] ? 1u << 16 : 0u);
        }
        // block exclusive scan of the packed (keep | merge << 16) counts
        uint32_t x = c;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t excl = x - c, total = 0;
        for (int v = 0; v < kPlocSmallThreads / 64; ++v) {
            const uint32_t t = wsum[v];
            if (v < w) excl += t;
            total += t;
        }
        float4 alo[kPlocPer], ahi[kPlocPer], blo[kPlocPer], bhi[kPlocPer];
        int2 ast[kPlocPer], bst[kPlocPer];
        for (int q = 0; q < kPlocPer; ++q) {
            const int i = i0 + q;
            if (i < m) {
                alo[q] = slo[i];
                ahi[q] = shi[i];
                ast[q] = sst[i];
                if (mf[q]) {
                    const int j = snn[i];
                    blo[q] = slo[j];
                    bhi[q] = shi[j];
                    bst[q] = sst[j];
                }
            }
        }
        __syncthreads();
        int kp = static_cast<int>(excl & 0xffffu), mp = static_cast<int>(excl >> 16);
        for (int q = 0; q < kPlocPer; ++q) {
            if (mf[q]) {
                if (node_base + mp < n_int) {
                    float4 ol, oh;
                    sst[kp] = ploc_merge(node_base + mp, alo[q], ahi[q], ast[q], blo[q], bhi[q], bst[q], nd, leaf_max,
                                         ol, oh);
                    slo[kp] = ol;
                    shi[kp] = oh;
                } else {
                    *err = 4;
                }
                ++kp;
                ++mp;
            } else if (kf[q]) {
                slo[kp] = alo[q];
                shi[kp] = ahi[q];
                sst[kp] = ast[q];
                ++kp;
            }
        }
        __syncthreads();
        m = static_cast<int>(total & 0xffffu);
        node_base += static_cast<int>(total >> 16);
    }
    if (tid == 0 && m != 1) *err = 2;
}

// Preorder index of every kept internal node (-1 for nodes inside a leaf),
// the first leaf slot of every internal node, and the leaf slot of every
// triangle: a walk to the root adds, for each step down to a right child,
// the left sibling's triangle count (slot) and kept-node count plus one
// (preorder), and one for each step down to a left child.
__global__ void k_ploc_walk(int n_int, int n, PlocNodes nd, int *__restrict__ pre, int *__restrict__ first,
                            int *__restrict__ slot_of, int *__restrict__ depth, int *__restrict__ err)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_int + n) return;
    const bool leaf = x >= n_int;
    const int id = leaf ? x - n_int : x;
    int par = leaf ? nd.pleaf[id] : nd.pint[id];
    bool kept = !leaf && nd.kept[id] > 0;
    int p_idx = 0, f_idx = 0, dep = 0;
    while (par >= 0) {
        const int p = par >> 1;
        if (p >= n_int || dep >= n) {
            *err = 3;
            break;
        }
        if (nd.kept[p] == 0) kept = false;
        if (par & 1) {
            const int l = nd.ch[p].x;
            if (l >= n_int || ~l >= n) {
                *err = 3;
                break;
            }
            f_idx += l < 0 ? 1 : __float_as_int(nd.hi[l].w);
            p_idx += 1 + (l < 0 ? 0 : nd.kept[l]);
        } else {
            p_idx += 1;
        }
        ++dep;
        par = nd.pint[p];
    }
    if (leaf) {
        slot_of[id] = f_idx;
    } else {
        pre[id] = kept ? p_idx : -1;
        first[id] = f_idx;
        if (kept) atomicMax(depth, dep + 1);
    }
}

// Kept internal nodes in preorder, both child boxes in the parent.
__global__ void k_ploc_emit(int n_int, int n, PlocNodes nd, const float *__restrict__ lbox,
                            const int *__restrict__ pre, const int *__restrict__ first,
                            const int *__restrict__ slot_of, BNode *__restrict__ out, int *__restrict__ err)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_int) return;
    const int q = pre[x];
    if (q < 0) return;
    const int2 cc = nd.ch[x];
    const int c[2] = {cc.x, cc.y};
    if (q >= n_int || c[0] >= n_int || c[1] >= n_int || ~c[0] >= n || ~c[1] >= n) {
        *err = 5;
        return;
    }
    float bx[2][6];
    int ref[2];
    for (int s = 0; s < 2; ++s) {
        if (c[s] < 0) {
            const float *b = lbox + 6 * (~c[s]);
            for (int k = 0; k < 6; ++k) bx[s][k] = b[k];
            ref[s] = leaf_ref(slot_of[~c[s]], 1);
        } else {
            const float4 l = nd.lo[c[s]], h = nd.hi[c[s]];
            bx[s][0] = l.x;
            bx[s][1] = l.y;
            bx[s][2] = l.z;
            bx[s][3] = h.x;
            bx[s][4] = h.y;
            bx[s][5] = h.z;
            ref[s] = nd.kept[c[s]] == 0 ? leaf_ref(first[c[s]], __float_as_int(h.w)) : pre[c[s]];
        }
    }
    BNode o;
    o.a = make_float4(bx[0][0], bx[0][1], bx[0][2], bx[0][3]);
    o.b = make_float4(bx[0][4], bx[0][5], bx[1][0], bx[1][1]);
    o.c = make_float4(bx[1][2], bx[1][3], bx[1][4], bx[1][5]);
    o.ch = make_int4(ref[0], ref[1], 0, 0);
    out[q] = o;
}

// Scratch arrays of one build, from the device block cache; handed back when
// the build returns (after its stream has drained: a successful build
// synchronises it, an error path returns early and the device is synchronised).
struct Temp {
    int device = 0;
    bool synced = false;  // the build's stream was synchronised after its last launch
    std::vector<std::pair<void *, size_t>> blocks;
    ~Temp()
    {
        if (blocks.empty()) return;
        if (!synced) (void)hipDeviceSynchronize();
        for (const auto &b : blocks) device_block_put(device, b.first, b.second);
    }
    template <class T>
    int alloc(T **p, size_t n)
    {
        size_t cap = 0;
        void *q = nullptr;
        const int rc = device_block_get(device, sizeof(T) * (n ? n : 1), &q, &cap);
        if (rc == SBR_OK) {
            *p = static_cast<T *>(q);
            blocks.emplace_back(q, cap);
        }
        return rc;
    }
};

inline unsigned blocks_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

namespace {

// Steps shared by both GPU builders: normals by input id, the live
// triangles on the device, the Morton sort, padded leaf boxes in sorted
// order.  done is set when no hierarchy is needed (no live triangle, or one
// leaf holds them all).
struct Front {
    int n = 0;
    float *v0 = nullptr, *e1 = nullptr, *e2 = nullptr, *nrm = nullptr, *lbox = nullptr;
    int32_t *ids = nullptr;
    uint64_t *keys = nullptr;   // sorted Morton codes
    uint32_t *order = nullptr;  // live index at each sorted position
    bool done = false;
};

int build_front(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, bool cubic, sbr_bvh *bvh, Temp &tmp,
                Front &f)
{
    if (leaf_max < 1 || leaf_max > kLeafMaxLimit) return fail(SBR_ERR_INVALID_ARG, "leaf size must be in [1, 4]");
    hipStream_t s = ctx->stream;
    const int64_t nt = bvh->n_tris;
    const int n = static_cast<int>(pm.live.size());
    f.n = n;
    int rc;
    std::vector<float4> nid(nt);
    for (int64_t j = 0; j < nt; ++j) nid[j] = make_float4(pm.n[3 * j], pm.n[3 * j + 1], pm.n[3 * j + 2], 0.f);
    if ((rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nrm_id), sizeof(float4) * (nt ? nt : 1)))) return rc;
    bvh->n_live = n;
    if (n == 0) {
        bvh->n_nodes = 0;
        bvh->depth = 0;
        f.done = true;
        if ((rc = upload_async(ctx, {{bvh->nrm_id, nid.data(), sizeof(float4) * nt}}))) return rc;
        SBR_HIP(hipStreamSynchronize(s));
        return SBR_OK;
    }
    // live triangle arrays, with the normals by id, through the pinned staging buffer
    std::vector<float> hv0(3 * n), he1(3 * n), he2(3 * n), hn(3 * n);
    for (int i = 0; i < n; ++i) {
        const int32_t j = pm.live[i];
        for (int a = 0; a < 3; ++a) {
            hv0[3 * i + a] = pm.v0[3 * j + a];
            he1[3 * i + a] = pm.e1[3 * j + a];
            he2[3 * i + a] = pm.e2[3 * j + a];
            hn[3 * i + a] = pm.n[3 * j + a];
        }
    }
    if ((rc = tmp.alloc(&f.v0, 3 * n)) || (rc = tmp.alloc(&f.e1, 3 * n)) || (rc = tmp.alloc(&f.e2, 3 * n)) ||
        (rc = tmp.alloc(&f.nrm, 3 * n)) || (rc = tmp.alloc(&f.ids, n)))
        return rc;
    if ((rc = upload_async(ctx, {{bvh->nrm_id, nid.data(), sizeof(float4) * nt},
                                 {f.v0, hv0.data(), 12 * static_cast<size_t>(n)},
                                 {f.e1, he1.data(), 12 * static_cast<size_t>(n)},
                                 {f.e2, he2.data(), 12 * static_cast<size_t>(n)},
                                 {f.nrm, hn.data(), 12 * static_cast<size_t>(n)},
                                 {f.ids, pm.live.data(), 4 * static_cast<size_t>(n)}})))
        return rc;

    // 1. Morton codes over the scene box
    uint64_t *k0, *k1;
    uint32_t *v0i, *v1i;
    if ((rc = tmp.alloc(&k0, n)) || (rc = tmp.alloc(&k1, n)) || (rc = tmp.alloc(&v0i, n)) ||
        (rc = tmp.alloc(&v1i, n)))
        return rc;
    // per-axis scale (LBVH), or one scale for all axes (PLOC: cube cells keep
    // the curve's neighbourhoods isotropic on elongated meshes)
    float lo[3], sc[3];
    double ext_max = 0.0;
    for (int a = 0; a < 3; ++a) ext_max = std::max(ext_max, pm.bbox[3 + a] - pm.bbox[a]);
    for (int a = 0; a < 3; ++a) {
        lo[a] = static_cast<float>(pm.bbox[a]);
        const double ext = cubic ? ext_max : pm.bbox[3 + a] - pm.bbox[a];
        sc[a] = ext > 0.0 ? static_cast<float>(2097152.0 / ext) : 0.0f;
    }
    k_morton<<<blocks_for(n, 256), 256, 0, s>>>(f.v0, f.e1, f.e2, n, lo[0], lo[1], lo[2], sc[0], sc[1], sc[2], k0,
                                                 v0i);
    SBR_HIP(hipGetLastError());

    // 2. sort: one workgroup for small meshes, else radix sort, 8 passes of 8 bits
    uint64_t *kin = k0, *kout = k1;
    uint32_t *vin = v0i, *vout = v1i;
    if (n <= kSmallSort) {
        k_sort_small<<<1, kSmallSort / 2, 0, s>>>(k0, v0i, n, k1, v1i);
        SBR_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    } else {
        const int nb = static_cast<int>(blocks_for(n, kSortTile));
        uint32_t *hist;
        if ((rc = tmp.alloc(&hist, static_cast<size_t>(256) * nb))) return rc;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 8 * pass;
            k_hist<<<nb, kSortThreads, 0, s>>>(kin, n, shift, hist, nb);
            k_scan<<<1, 1024, 0, s>>>(hist, 256 * nb);
            k_scatter<<<nb, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, shift, hist, nb);
            SBR_HIP(hipGetLastError());
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
    }
    f.keys = kin;
    f.order = vin;

    // padded leaf boxes; the BVH's triangle arrays
    const int n_int = std::max(1, n - 1);
    if ((rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nodes), sizeof(BNode) * n_int)) ||
        (rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->tris), sizeof(BTri) * n)) ||
        (rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nrm_slot), sizeof(float4) * n)) ||
        (rc = tmp.alloc(&f.lbox, 6 * static_cast<size_t>(n))))
        return rc;
    const SceneScale scl = scene_scale(pm.bbox, pm.diag);
    k_leaf_boxes<<<blocks_for(n, 256), 256, 0, s>>>(n, f.order, f.v0, f.e1, f.e2, scl.pbox, scl.guard, f.lbox);
    SBR_HIP(hipGetLastError());
    if (n <= leaf_max) {
        k_place<<<blocks_for(n, 256), 256, 0, s>>>(n, f.order, nullptr, f.v0, f.e1, f.e2, f.nrm, f.ids, bvh->tris,
                                                   bvh->nrm_slot);
        k_single<<<1, 1, 0, s>>>(n, f.lbox, bvh->nodes);
        SBR_HIP(hipGetLastError());
        SBR_HIP(hipStreamSynchronize(s));
        tmp.synced = true;
        bvh->n_nodes = 1;
        bvh->depth = 1;
        f.done = true;
    }
    return SBR_OK;
}

}  // namespace

int build_lbvh(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh)
{
    hipStream_t s = ctx->stream;
    Temp tmp;
    tmp.device = ctx->device;
    Front f;
    int rc = build_front(ctx, pm, leaf_max, false, bvh, tmp, f);
    if (rc || f.done) return rc;
    const int n = f.n, n_int = n - 1;

    // 3-5. hierarchy, refit, preorder relayout
    k_place<<<blocks_for(n, 256), 256, 0, s>>>(n, f.order, nullptr, f.v0, f.e1, f.e2, f.nrm, f.ids, bvh->tris,
                                               bvh->nrm_slot);
    int *left, *right, *pint, *pleaf, *rfirst, *rlast, *arrive, *pre, *depth;
    uint32_t *newidx;
    uint8_t *isleft;
    float *nbox;
    if ((rc = tmp.alloc(&left, n_int)) || (rc = tmp.alloc(&right, n_int)) || (rc = tmp.alloc(&pint, n_int)) ||
        (rc = tmp.alloc(&pleaf, n)) || (rc = tmp.alloc(&rfirst, n_int)) || (rc = tmp.alloc(&rlast, n_int)) ||
        (rc = tmp.alloc(&arrive, n_int)) || (rc = tmp.alloc(&pre, n_int)) || (rc = tmp.alloc(&depth, 1)) ||
        (rc = tmp.alloc(&isleft, n_int)) || (rc = tmp.alloc(&newidx, n_int + 1)) ||
        (rc = tmp.alloc(&nbox, 6 * static_cast<size_t>(n_int))))
        return rc;
    SBR_HIP(hipMemsetAsync(arrive, 0, sizeof(int) * n_int, s));
    SBR_HIP(hipMemsetAsync(depth, 0, sizeof(int), s));
    SBR_HIP(hipMemsetAsync(isleft, 0, n_int, s));
    SBR_HIP(hipMemsetAsync(newidx, 0, sizeof(uint32_t) * (n_int + 1), s));
    k_karras<<<blocks_for(n_int, 256), 256, 0, s>>>(f.keys, n, left, right, pint, pleaf, rfirst, rlast, isleft);
    k_refit<<<blocks_for(n, 256), 256, 0, s>>>(n, left, right, pint, pleaf, f.lbox, nbox, arrive);
    k_preorder<<<blocks_for(n_int, 256), 256, 0, s>>>(n_int, pint, isleft, rfirst, pre, depth);
    k_mark_kept<<<blocks_for(n_int, 256), 256, 0, s>>>(n_int, pre, rfirst, rlast, leaf_max, newidx);
    k_scan<<<1, 1024, 0, s>>>(newidx, n_int + 1);  // newidx[n_int] becomes the kept-node count
    k_relayout<<<blocks_for(n_int, 256), 256, 0, s>>>(n_int, left, right, pre, newidx, rfirst, rlast, leaf_max, f.lbox,
                                                      nbox, bvh->nodes);
    SBR_HIP(hipGetLastError());
    int hdepth = 0;
    uint32_t kept = 0;
    SBR_HIP(hipMemcpyAsync(&hdepth, depth, sizeof(int), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipMemcpyAsync(&kept, newidx + n_int, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    tmp.synced = true;
    bvh->depth = hdepth;
    bvh->n_nodes = kept;
    return SBR_OK;
}

int build_ploc(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh)
{
    hipStream_t s = ctx->stream;
    Temp tmp;
    tmp.device = ctx->device;
    Front f;
    int rc = build_front(ctx, pm, leaf_max, true, bvh, tmp, f);
    if (rc || f.done) return rc;
    const int n = f.n, n_int = n - 1;
    const int n_tiles = static_cast<int>(blocks_for(n, kPlocTile));

    float4 *clo[2], *chi[2];
    int *nn, *pre, *first, *slot_of, *flags;  // flags: [0] depth, [1] error
    uint2 *tc;
    PlocState *st;
    PlocNodes nd;
    if ((rc = tmp.alloc(&clo[0], n)) || (rc = tmp.alloc(&clo[1], n)) || (rc = tmp.alloc(&chi[0], n)) ||
        (rc = tmp.alloc(&chi[1], n)) || (rc = tmp.alloc(&nn, n)) || (rc = tmp.alloc(&tc, n_tiles)) ||
        (rc = tmp.alloc(&st, 2)) || (rc = tmp.alloc(&flags, 2)) || (rc = tmp.alloc(&nd.lo, n_int)) ||
        (rc = tmp.alloc(&nd.hi, n_int)) || (rc = tmp.alloc(&nd.ch, n_int)) || (rc = tmp.alloc(&nd.kept, n_int)) ||
        (rc = tmp.alloc(&nd.pint, n_int)) || (rc = tmp.alloc(&nd.pleaf, n)) || (rc = tmp.alloc(&pre, n_int)) ||
        (rc = tmp.alloc(&first, n_int)) || (rc = tmp.alloc(&slot_of, n)))
        return rc;
    SBR_HIP(hipMemsetAsync(nd.pint, 0xff, sizeof(int) * n_int, s));  // the root keeps -1
    SBR_HIP(hipMemsetAsync(flags, 0, 2 * sizeof(int), s));
    k_ploc_init<<<blocks_for(n, 256), 256, 0, s>>>(n, f.lbox, clo[0], chi[0], st);
    SBR_HIP(hipGetLastError());

    // steps over the whole cluster array until kPlocSmall clusters are left;
    // the host reads the count every fourth step (launch grids follow the
    // last count read; the kernels use the count on the device)
    int m = n, t = 0;
    while (m > kPlocSmall) {
        const unsigned g = blocks_for(m, kPlocTile);
        const PlocState *cur = st + (t & 1);
        PlocState *nxt = st + ((t + 1) & 1);
        k_ploc_nn<<<g, kPlocTile, 0, s>>>(cur, clo[t & 1], chi[t & 1], nn);
        k_ploc_count<<<g, kPlocTile, 0, s>>>(cur, nn, tc);
        k_ploc_scan<<<1, 1024, 0, s>>>(cur, nxt, tc);
        k_ploc_apply<<<g, kPlocTile, 0, s>>>(cur, nn, tc, clo[t & 1], chi[t & 1], clo[(t + 1) & 1], chi[(t + 1) & 1],
                                             nd, leaf_max, n_int, flags + 1);
        SBR_HIP(hipGetLastError());
        ++t;
        if ((t & 3) == 0) {
            PlocState h;
            SBR_HIP(hipMemcpyAsync(&h, st + (t & 1), sizeof(h), hipMemcpyDeviceToHost, s));
            SBR_HIP(hipStreamSynchronize(s));
            if (h.m >= m || h.m < 1) return fail(SBR_ERR_HIP, "PLOC build: the cluster count did not shrink");
            m = h.m;
        }
        if (t > kPlocMaxSteps) return fail(SBR_ERR_HIP, "PLOC build: too many steps");
    }
    k_ploc_small<<<1, kPlocSmallThreads, 0, s>>>(st + (t & 1), clo[t & 1], chi[t & 1], nd, leaf_max, n_int,
                                                 flags + 1);
    SBR_HIP(hipGetLastError());

    // layout: preorder indices and leaf slots, the kept nodes, the triangles
    // (every index these kernels follow is range-checked, so a failed
    // clustering is reported through the flags instead of faulting)
    k_ploc_walk<<<blocks_for(static_cast<int64_t>(n_int) + n, 256), 256, 0, s>>>(n_int, n, nd, pre, first, slot_of,
                                                                                 flags, flags + 1);
    k_ploc_emit<<<blocks_for(n_int, 256), 256, 0, s>>>(n_int, n, nd, f.lbox, pre, first, slot_of, bvh->nodes,
                                                       flags + 1);
    k_place<<<blocks_for(n, 256), 256, 0, s>>>(n, f.order, slot_of, f.v0, f.e1, f.e2, f.nrm, f.ids, bvh->tris,
                                               bvh->nrm_slot);
    SBR_HIP(hipGetLastError());
    int kept = 0, hf[2] = {0, 0};
    SBR_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipMemcpyAsync(&kept, nd.kept + (n - 2), sizeof(int), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    tmp.synced = true;
    if (hf[1]) return fail(SBR_ERR_HIP, "PLOC build: clustering or layout failed (code " + std::to_string(hf[1]) + ")");
    if (kept < 1 || kept > n_int) return fail(SBR_ERR_HIP, "PLOC build: bad node count");
    bvh->depth = hf[0];
    bvh->n_nodes = kept;
    return SBR_OK;
}

}  // namespace sbr
