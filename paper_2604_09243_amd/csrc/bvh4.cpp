// Four-wide BVH collapsed from the binary layout that every builder emits.
//
// The binary tree (BNode: both child boxes inline) is the one the builders,
// the validator, the primary-ray mask and the multi-scene arena use; the
// trace kernels can instead walk this collapsed copy, which tests four child
// boxes per 128-byte fetch and so needs about half the dependent node fetches
// per query.  The collapse only regroups nodes: every child box of a BVH4 node
// is a child box of the BVH2, so it holds the same guard-widened triangle
// boxes and the traversal's exactness argument carries over unchanged (the
// closest hit is found whichever tree is walked; only the visiting order and
// the work differ).
//
// A BVH4 node starts from the two children of a BVH2 node and repeatedly
// opens (replaces by its two children) the internal candidate with the
// largest surface area until it holds four or no candidate is internal, the
// usual greedy collapse.  Nodes are numbered so that the internal children of
// a node are consecutive, the root at 0.
#include <algorithm>
#include <cstring>
#include <vector>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

struct Cand {
    int ref;
    float lo[3], hi[3];
};

Cand child_of(const BNode &n, int s)
{
    Cand c;
    if (s == 0) {
        c.ref = n.ch.x;
        c.lo[0] = n.a.x; c.lo[1] = n.a.y; c.lo[2] = n.a.z;
        c.hi[0] = n.a.w; c.hi[1] = n.b.x; c.hi[2] = n.b.y;
    } else {
        c.ref = n.ch.y;
        c.lo[0] = n.b.z; c.lo[1] = n.b.w; c.lo[2] = n.c.x;
        c.hi[0] = n.c.y; c.hi[1] = n.c.z; c.hi[2] = n.c.w;
    }
    return c;
}

double area(const Cand &c)
{
    const double dx = double(c.hi[0]) - c.lo[0], dy = double(c.hi[1]) - c.lo[1], dz = double(c.hi[2]) - c.lo[2];
    return dx * dy + dy * dz + dz * dx;
}

// The children of BVH2 node `n` (one for the single-leaf tree, whose node
// repeats its leaf).
int children(const BNode &n, Cand *c)
{
    c[0] = child_of(n, 0);
    if (n.ch.y == n.ch.x) return 1;
    c[1] = child_of(n, 1);
    return 2;
}

}  // namespace

int collapse_wide(const std::vector<BNode> &hn, std::vector<BNode4> &out, int &depth4)
{
    out.clear();
    depth4 = 0;
    if (hn.empty()) return SBR_OK;
    const int nn = static_cast<int>(hn.size());
    struct Work {
        int node2, node4, depth;
    };
    std::vector<Work> st;
    st.push_back({0, 0, 1});
    out.resize(1);
    while (!st.empty()) {
        const Work w = st.back();
        st.pop_back();
        depth4 = std::max(depth4, w.depth);
        if (w.node2 < 0 || w.node2 >= nn) return fail(SBR_ERR_INVALID_MESH, "BVH collapse: bad node reference");
        Cand c[4];
        int n = children(hn[w.node2], c);
        for (;;) {
            if (n >= 4) break;
            int best = -1;
            double best_a = -1.0;
            for (int i = 0; i < n; ++i)
                if (c[i].ref >= 0 && area(c[i]) > best_a) {
                    best_a = area(c[i]);
                    best = i;
                }
            if (best < 0) break;
            const int r = c[best].ref;
            if (r >= nn) return fail(SBR_ERR_INVALID_MESH, "BVH collapse: bad node reference");
            Cand g[2];
            if (children(hn[r], g) != 2) return fail(SBR_ERR_INVALID_MESH, "BVH collapse: inner node with one child");
            c[best] = g[0];
            c[n++] = g[1];
        }
        int n_inner = 0;
        for (int i = 0; i < n; ++i) n_inner += c[i].ref >= 0;
        const int base = static_cast<int>(out.size());
        out.resize(out.size() + n_inner);
        BNode4 &o = out[w.node4];
        std::memset(&o, 0, sizeof(o));
        float *lx = &o.lox.x, *hx = &o.hix.x, *ly = &o.loy.x, *hy = &o.hiy.x, *lz = &o.loz.x, *hz = &o.hiz.x;
        int *ch = &o.ch.x;
        int k = 0;
        for (int i = 0; i < 4; ++i) {
            const Cand &q = c[i < n ? i : 0];
            lx[i] = q.lo[0]; hx[i] = q.hi[0];
            ly[i] = q.lo[1]; hy[i] = q.hi[1];
            lz[i] = q.lo[2]; hz[i] = q.hi[2];
            if (i >= n) {
                ch[i] = kNoChild;
            } else if (q.ref >= 0) {
                ch[i] = base + k;
                st.push_back({q.ref, base + k, w.depth + 1});
                ++k;
            } else {
                ch[i] = q.ref;
            }
        }
        o.m.x = n;
    }
    return SBR_OK;
}

int validate_wide(const std::vector<BNode> &hn, const std::vector<BNode4> &w, int depth4)
{
    // the BVH4 holds exactly the leaves of the BVH2, each once and with the
    // box the BVH2 gives it (so the BVH2's leaf-box checks carry over), and
    // every internal child's boxes lie inside the box its parent gives it
    std::vector<std::pair<int, Cand>> leaves;  // (leaf code, box) of the BVH2
    for (const BNode &n : hn) {
        Cand c[2];
        const int k = children(n, c);
        for (int i = 0; i < k; ++i)
            if (c[i].ref < 0) leaves.push_back({~c[i].ref, c[i]});
    }
    std::sort(leaves.begin(), leaves.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (size_t i = 1; i < leaves.size(); ++i)
        if (leaves[i].first == leaves[i - 1].first) return fail(SBR_ERR_INVALID_MESH, "BVH layout: leaf in two nodes");
    std::vector<uint8_t> seen_leaf(leaves.size(), 0), seen(w.size(), 0);
    const int nw = static_cast<int>(w.size());
    if (nw == 0) return hn.empty() ? SBR_OK : fail(SBR_ERR_INVALID_MESH, "BVH4: no nodes");
    std::vector<std::pair<int, int>> st{{0, 1}};
    while (!st.empty()) {
        const int t = st.back().first, d = st.back().second;
        st.pop_back();
        if (t < 0 || t >= nw || seen[t]) return fail(SBR_ERR_INVALID_MESH, "BVH4: bad node reference");
        if (d > depth4) return fail(SBR_ERR_INVALID_MESH, "BVH4: depth bound");
        seen[t] = 1;
        const BNode4 &o = w[t];
        const int n = o.m.x;
        if (n < 1 || n > 4) return fail(SBR_ERR_INVALID_MESH, "BVH4: child count");
        const float *lx = &o.lox.x, *hx = &o.hix.x, *ly = &o.loy.x, *hy = &o.hiy.x, *lz = &o.loz.x, *hz = &o.hiz.x;
        const int *ch = &o.ch.x;
        for (int i = 0; i < 4; ++i) {
            if ((ch[i] == kNoChild) != (i >= n)) return fail(SBR_ERR_INVALID_MESH, "BVH4: absent child misplaced");
            if (i >= n) continue;
            const float lo[3] = {lx[i], ly[i], lz[i]}, hi[3] = {hx[i], hy[i], hz[i]};
            if (ch[i] >= 0) {
                if (ch[i] <= t || ch[i] >= nw) return fail(SBR_ERR_INVALID_MESH, "BVH4: child before parent");
                const BNode4 &c = w[ch[i]];
                for (int j = 0; j < c.m.x && j < 4; ++j) {
                    const float clo[3] = {(&c.lox.x)[j], (&c.loy.x)[j], (&c.loz.x)[j]};
                    const float chi[3] = {(&c.hix.x)[j], (&c.hiy.x)[j], (&c.hiz.x)[j]};
                    for (int k = 0; k < 3; ++k)
                        if (!(clo[k] >= lo[k] && chi[k] <= hi[k]))
                            return fail(SBR_ERR_INVALID_MESH, "BVH4: child box outside its parent");
                }
                st.push_back({ch[i], d + 1});
            } else {
                const int code = ~ch[i];
                auto it = std::lower_bound(leaves.begin(), leaves.end(), code,
                                           [](const auto &a, int v) { return a.first < v; });
                if (it == leaves.end() || it->first != code) return fail(SBR_ERR_INVALID_MESH, "BVH4: unknown leaf");
                const size_t q = static_cast<size_t>(it - leaves.begin());
                if (seen_leaf[q]) return fail(SBR_ERR_INVALID_MESH, "BVH4: leaf reached twice");
                seen_leaf[q] = 1;
                for (int k = 0; k < 3; ++k)
                    if (lo[k] != it->second.lo[k] || hi[k] != it->second.hi[k])
                        return fail(SBR_ERR_INVALID_MESH, "BVH4: leaf box differs from the BVH2's");
            }
        }
    }
    for (size_t q = 0; q < leaves.size(); ++q)
        if (!seen_leaf[q]) return fail(SBR_ERR_INVALID_MESH, "BVH4: leaf not reached");
    for (int t = 0; t < nw; ++t)
        if (!seen[t]) return fail(SBR_ERR_INVALID_MESH, "BVH4: unreachable node");
    return SBR_OK;
}

int build_wide(sbr_ctx *ctx, sbr_bvh *bvh)
{
    if (bvh->n_nodes <= 0 || bvh->nodes4) return SBR_OK;
    std::vector<BNode> hn(static_cast<size_t>(bvh->n_nodes));
    SBR_HIP(hipMemcpyAsync(hn.data(), bvh->nodes, sizeof(BNode) * hn.size(), hipMemcpyDeviceToHost, ctx->stream));
    SBR_HIP(hipStreamSynchronize(ctx->stream));
    std::vector<BNode4> w;
    int depth4 = 0;
    int rc = collapse_wide(hn, w, depth4);
    if (rc) return rc;
    if ((rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nodes4), sizeof(BNode4) * w.size()))) return rc;
    if ((rc = upload_async(ctx, {{bvh->nodes4, w.data(), sizeof(BNode4) * w.size()}}))) return rc;
    // the host vector is freed on return: wait for the staged copy
    SBR_HIP(hipStreamSynchronize(ctx->stream));
    bvh->n_nodes4 = static_cast<int64_t>(w.size());
    bvh->depth4 = depth4;
    return SBR_OK;
}

}  // namespace sbr
