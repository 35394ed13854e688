// GPU BVH construction (linear BVH).
//
// The paper builds a median / binned-SAH BVH recursively on the host
// (Sec. 4, Algorithm 1).  Here the tree is built on the device in a fixed
// number of data-parallel passes:
//   1. 63-bit Morton code of each triangle centroid (21 bits per axis);
//   2. stable LSD radix sort of (code, triangle) in eight 8-bit passes, each
//      pass a per-tile LDS histogram, one scan of all tile histograms, and an
//      LDS-ranked scatter (wave ballots give the rank among equal digits);
//   3. the radix-tree hierarchy over the sorted codes (one thread per
//      internal node, longest-common-prefix split search; equal codes are
//      separated by their sorted index);
//   4. bottom-up refit of padded boxes: one thread per leaf climbs towards
//      the root and stops at the first parent whose other child is not done
//      yet (per-node arrival counter);
//   5. relayout into preorder, with both child boxes stored in the parent.
// Subtrees of at most leaf_max triangles are collapsed into leaves (their
// triangles are contiguous in sorted order), the leaf threshold of the
// paper's build.  Boxes are padded so the traversal's box test never culls a
// triangle the float32 intersection test would accept.
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

// Triangles in sorted (leaf) order, their normals, and padded leaf boxes.
__global__ void k_leaves(int n, const uint32_t *__restrict__ order, const float *__restrict__ v0,
                         const float *__restrict__ e1, const float *__restrict__ e2, const float *__restrict__ nrm,
                         const int32_t *__restrict__ ids, float pad, BTri *__restrict__ tris,
                         float4 *__restrict__ nrm_slot, float *__restrict__ lbox)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int li = static_cast<int>(order[j]);
    const float *a = v0 + 3 * li, *b = e1 + 3 * li, *c = e2 + 3 * li;
    BTri t;
    t.p0 = make_float4(a[0], a[1], a[2], __int_as_float(ids[li]));
    t.p1 = make_float4(b[0], b[1], b[2], 0.0f);
    t.p2 = make_float4(c[0], c[1], c[2], 0.0f);
    tris[j] = t;
    nrm_slot[j] = make_float4(nrm[3 * li], nrm[3 * li + 1], nrm[3 * li + 2], 0.0f);
    for (int k = 0; k < 3; ++k) {
        const float p0 = a[k], p1 = a[k] + b[k], p2 = a[k] + c[k];
        const float lo = fminf(p0, fminf(p1, p2)), hi = fmaxf(p0, fmaxf(p1, p2));
        lbox[6 * j + k] = lo - pad - fabsf(lo) * 4e-7f;
        lbox[6 * j + 3 + k] = hi + pad + fabsf(hi) * 4e-7f;
    }
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

// Scratch arrays of one build, from the device block cache; handed back when
// the build returns (after the device is idle: error paths return early).
struct Temp {
    int device = 0;
    std::vector<std::pair<void *, size_t>> blocks;
    ~Temp()
    {
        if (blocks.empty()) return;
        (void)hipDeviceSynchronize();
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

int build_lbvh(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh)
{
    if (leaf_max < 1 || leaf_max > kLeafMaxLimit) return fail(SBR_ERR_INVALID_ARG, "leaf size must be in [1, 4]");
    hipStream_t s = ctx->stream;
    const int64_t nt = bvh->n_tris;
    const int n = static_cast<int>(pm.live.size());
    Temp tmp;
    tmp.device = ctx->device;
    int rc;
    // normals by input id (float4) for the PO stage
    {
        std::vector<float4> nid(nt);
        for (int64_t j = 0; j < nt; ++j) nid[j] = make_float4(pm.n[3 * j], pm.n[3 * j + 1], pm.n[3 * j + 2], 0.f);
        if ((rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nrm_id), sizeof(float4) * (nt ? nt : 1)))) return rc;
        SBR_HIP(hipMemcpy(bvh->nrm_id, nid.data(), sizeof(float4) * nt, hipMemcpyHostToDevice));
    }
    bvh->n_live = n;
    if (n == 0) {
        bvh->n_nodes = 0;
        bvh->depth = 0;
        return SBR_OK;
    }
    // live triangle arrays
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
    float *dv0, *de1, *de2, *dn;
    int32_t *dids;
    if ((rc = tmp.alloc(&dv0, 3 * n)) || (rc = tmp.alloc(&de1, 3 * n)) || (rc = tmp.alloc(&de2, 3 * n)) ||
        (rc = tmp.alloc(&dn, 3 * n)) || (rc = tmp.alloc(&dids, n)))
        return rc;
    SBR_HIP(hipMemcpyAsync(dv0, hv0.data(), 12 * n, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(de1, he1.data(), 12 * n, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(de2, he2.data(), 12 * n, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dn, hn.data(), 12 * n, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dids, pm.live.data(), 4 * n, hipMemcpyHostToDevice, s));

    // 1. Morton codes over the scene box
    uint64_t *k0, *k1;
    uint32_t *v0i, *v1i;
    if ((rc = tmp.alloc(&k0, n)) || (rc = tmp.alloc(&k1, n)) || (rc = tmp.alloc(&v0i, n)) ||
        (rc = tmp.alloc(&v1i, n)))
        return rc;
    float lo[3], sc[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = static_cast<float>(pm.bbox[a]);
        const double ext = pm.bbox[3 + a] - pm.bbox[a];
        sc[a] = ext > 0.0 ? static_cast<float>(2097152.0 / ext) : 0.0f;
    }
    k_morton<<<blocks_for(n, 256), 256, 0, s>>>(dv0, de1, de2, n, lo[0], lo[1], lo[2], sc[0], sc[1], sc[2], k0,
                                                 v0i);
    SBR_HIP(hipGetLastError());

    // 2. radix sort, 8 passes of 8 bits
    const int nb = static_cast<int>(blocks_for(n, kSortTile));
    uint32_t *hist;
    if ((rc = tmp.alloc(&hist, static_cast<size_t>(256) * nb))) return rc;
    uint64_t *kin = k0, *kout = k1;
    uint32_t *vin = v0i, *vout = v1i;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        k_hist<<<nb, kSortThreads, 0, s>>>(kin, n, shift, hist, nb);
        k_scan<<<1, 1024, 0, s>>>(hist, 256 * nb);
        k_scatter<<<nb, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, shift, hist, nb);
        SBR_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }

    // 3-5. hierarchy, leaves, refit, preorder relayout
    const int n_int = std::max(1, n - 1);
    bvh->n_nodes = n_int;
    if ((rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nodes), sizeof(BNode) * n_int)) ||
        (rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->tris), sizeof(BTri) * n)) ||
        (rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nrm_slot), sizeof(float4) * n)))
        return rc;
    float *lbox;
    if ((rc = tmp.alloc(&lbox, 6 * static_cast<size_t>(n)))) return rc;
    const float pad = static_cast<float>(1e-6 * pm.diag) + 1e-30f;
    k_leaves<<<blocks_for(n, 256), 256, 0, s>>>(n, vin, dv0, de1, de2, dn, dids, pad, bvh->tris, bvh->nrm_slot,
                                                lbox);
    SBR_HIP(hipGetLastError());
    if (n <= leaf_max) {
        k_single<<<1, 1, 0, s>>>(n, lbox, bvh->nodes);
        SBR_HIP(hipGetLastError());
        SBR_HIP(hipStreamSynchronize(s));
        bvh->n_nodes = 1;
        bvh->depth = 1;
        return SBR_OK;
    }
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
    k_karras<<<blocks_for(n_int, 256), 256, 0, s>>>(kin, n, left, right, pint, pleaf, rfirst, rlast, isleft);
    k_refit<<<blocks_for(n, 256), 256, 0, s>>>(n, left, right, pint, pleaf, lbox, nbox, arrive);
    k_preorder<<<blocks_for(n_int, 256), 256, 0, s>>>(n_int, pint, isleft, rfirst, pre, depth);
    k_mark_kept<<<blocks_for(n_int, 256), 256, 0, s>>>(n_int, pre, rfirst, rlast, leaf_max, newidx);
    k_scan<<<1, 1024, 0, s>>>(newidx, n_int + 1);  // newidx[n_int] becomes the kept-node count
    k_relayout<<<blocks_for(n_int, 256), 256, 0, s>>>(n_int, left, right, pre, newidx, rfirst, rlast, leaf_max, lbox, nbox,
                                                      bvh->nodes);
    SBR_HIP(hipGetLastError());
    int hdepth = 0;
    uint32_t kept = 0;
    SBR_HIP(hipMemcpyAsync(&hdepth, depth, sizeof(int), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipMemcpyAsync(&kept, newidx + n_int, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SBR_HIP(hipStreamSynchronize(s));
    bvh->depth = hdepth;
    bvh->n_nodes = kept;
    return SBR_OK;
}

}  // namespace sbr
