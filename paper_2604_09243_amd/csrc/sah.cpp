// Host binned-SAH BVH builder (the top-down surface-area split of the
// paper's Algorithm 1 and its SAH cost), emitting exactly the node and
// triangle layout of the GPU LBVH so that the same traversal kernels run on
// it: nodes in preorder with the root at 0, both child boxes inline, leaves
// of at most leaf_max triangles coded ~(first * 8 + count - 1), triangles in
// leaf order.  Boxes are the same padded float32 triangle boxes as the LBVH
// (pad = 1e-6 |diag| plus 4e-7 of the coordinate), so the box test stays
// conservative.
//
// Split choice per node: 32 bins of the centroid extent on each axis; the
// cost of a split is C_node + (A_L n_L + A_R n_R) / A with C_node = 1.5 (one
// node visit, both child boxes, measured at about 1.5 triangle tests of the
// trace kernel); a node becomes a leaf when it holds at most leaf_max triangles and
// no split is cheaper than testing them all; a node whose centroids coincide
// splits at the middle index.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sbr_internal.hpp"

namespace sbr {
namespace {

constexpr int kBins = 32;
static_assert(kBins <= 32, "bin occupancy is a 32-bit mask");
// A node visit (both child boxes) costs about 1.5 triangle tests in the
// trace kernel (stack and loop work, lanes diverging between the two
// phases, while a leaf's triangles are tested together): 0.5, 1.0, 1.5 and
// 2.0 measured on the 64-scene batch at 2.56, 2.43, 2.36 and 2.32 s, with
// the trihedral's tree the same up to 1.5 and slower at 2.0.
constexpr float kNodeCost = 1.5f;

struct Box {
    float lo[3], hi[3];
    void empty()
    {
        for (int k = 0; k < 3; ++k) {
            lo[k] = INFINITY;
            hi[k] = -INFINITY;
        }
    }
    void grow(const Box &b)
    {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    float area() const
    {
        const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        if (!(dx >= 0.f)) return 0.f;
        return 2.f * (dx * dy + dy * dz + dz * dx);
    }
};

struct TNode {
    Box box;
    int left = -1, right = -1;  // tree children (internal) or -1
    int first = 0, count = 0;   // leaf range (count > 0)
};

struct Builder {
    const std::vector<Box> &pb;
    const std::vector<float> &cen;  // [n][3]
    std::vector<int> &idx;
    int leaf_max;
    std::vector<TNode> nodes;
    int depth = 0;

    Builder(const std::vector<Box> &b, const std::vector<float> &c, std::vector<int> &i, int lm)
        : pb(b), cen(c), idx(i), leaf_max(lm) {}

    int make_leaf(int b, int e, const Box &box)
    {
        TNode t;
        t.box = box;
        t.first = b;
        t.count = e - b;
        nodes.push_back(t);
        return static_cast<int>(nodes.size()) - 1;
    }

    // builds the subtree of idx[b, e); returns its node
    int build(int b, int e, int d)
    {
        depth = std::max(depth, d);
        Box box, cb;
        box.empty();
        cb.empty();
        for (int i = b; i < e; ++i) {
            box.grow(pb[idx[i]]);
            const float *c = &cen[3 * idx[i]];
            for (int k = 0; k < 3; ++k) {
                cb.lo[k] = std::min(cb.lo[k], c[k]);
                cb.hi[k] = std::max(cb.hi[k], c[k]);
            }
        }
        const int n = e - b;
        if (n == 1) return make_leaf(b, e, box);
        // best binned split over the three axes: one pass bins every
        // triangle on all axes, then each axis sweeps only its occupied bins
        // (an empty bin changes neither side of a split, so the costs, and
        // the first minimum, are those of a sweep over all kBins)
        float best = INFINITY;
        int best_axis = -1, best_bin = -1;
        const float parent_area = std::max(box.area(), 1e-30f);
        float sc[3];
        bool ok[3];
        for (int ax = 0; ax < 3; ++ax) {
            const float ext = cb.hi[ax] - cb.lo[ax];
            ok[ax] = ext > 0.f;
            sc[ax] = ok[ax] ? kBins / ext : 0.f;
        }
        Box bb[3][kBins];
        int bc[3][kBins];
        uint32_t occ[3] = {0u, 0u, 0u};
        for (int i = b; i < e; ++i) {
            const int t = idx[i];
            for (int ax = 0; ax < 3; ++ax) {
                if (!ok[ax]) continue;
                int q = static_cast<int>((cen[3 * t + ax] - cb.lo[ax]) * sc[ax]);
                q = std::min(std::max(q, 0), kBins - 1);
                if (occ[ax] >> q & 1u) {
                    bb[ax][q].grow(pb[t]);
                    ++bc[ax][q];
                } else {
                    occ[ax] |= 1u << q;
                    bb[ax][q] = pb[t];
                    bc[ax][q] = 1;
                }
            }
        }
        for (int ax = 0; ax < 3; ++ax) {
            if (!ok[ax]) continue;
            int qs[kBins], m = 0;
            for (uint32_t bits = occ[ax]; bits; bits &= bits - 1) qs[m++] = __builtin_ctz(bits);
            float ra[kBins];
            int rn[kBins];
            Box acc;
            acc.empty();
            int cnt = 0;
            for (int j = m - 1; j >= 1; --j) {
                acc.grow(bb[ax][qs[j]]);
                cnt += bc[ax][qs[j]];
                ra[j] = acc.area();
                rn[j] = cnt;
            }
            acc.empty();
            cnt = 0;
            for (int j = 0; j < m - 1; ++j) {
                acc.grow(bb[ax][qs[j]]);
                cnt += bc[ax][qs[j]];
                const float cost = kNodeCost + (acc.area() * cnt + ra[j + 1] * rn[j + 1]) / parent_area;
                if (cost < best) {
                    best = cost;
                    best_axis = ax;
                    best_bin = qs[j];
                }
            }
        }
        if (n <= leaf_max && !(best < static_cast<float>(n))) return make_leaf(b, e, box);
        int mid;
        if (best_axis < 0) {
            mid = b + n / 2;  // coincident centroids: split by index
        } else {
            const float ext = cb.hi[best_axis] - cb.lo[best_axis];
            const float sc = kBins / ext;
            auto it = std::partition(idx.begin() + b, idx.begin() + e, [&](int t) {
                int q = static_cast<int>((cen[3 * t + best_axis] - cb.lo[best_axis]) * sc);
                q = std::min(std::max(q, 0), kBins - 1);
                return q <= best_bin;
            });
            mid = static_cast<int>(it - idx.begin());
            if (mid == b || mid == e) mid = b + n / 2;
        }
        const int me = static_cast<int>(nodes.size());
        nodes.push_back(TNode());
        nodes[me].box = box;
        const int l = build(b, mid, d + 1);
        const int r = build(mid, e, d + 1);
        nodes[me].left = l;
        nodes[me].right = r;
        return me;
    }
};

void put_child(BNode &bn, int s, const Box &b)
{
    float *f = reinterpret_cast<float *>(&bn);  // a, b, c: 12 floats, child 0 then child 1
    for (int k = 0; k < 3; ++k) {
        f[6 * s + k] = b.lo[k];
        f[6 * s + 3 + k] = b.hi[k];
    }
}

}  // namespace

int sah_layout(const PreparedMesh &pm, int leaf_max, std::vector<BNode> &hn, std::vector<BTri> &ht,
               std::vector<float4> &hs, int &depth)
{
    const int n = static_cast<int>(pm.live.size());
    // triangle boxes (the hit rule's box widened by the guard: the same float32
    // arithmetic as the LBVH leaves) and centroids
    const SceneScale sc = scene_scale(pm.bbox, pm.diag);
    std::vector<Box> pb(n);
    std::vector<float> cen(3 * static_cast<size_t>(n));
    for (int j = 0; j < n; ++j) {
        const int li = pm.live[j];
        const float *a = &pm.v0[3 * li], *b = &pm.e1[3 * li], *c = &pm.e2[3 * li];
        for (int k = 0; k < 3; ++k) {
            float lo, hi;
            spec_box_axis(a[k], b[k], c[k], sc.pbox, lo, hi);
            pb[j].lo[k] = lo - sc.guard;
            pb[j].hi[k] = hi + sc.guard;
            cen[3 * j + k] = 0.5f * (pb[j].lo[k] + pb[j].hi[k]);
        }
    }
    std::vector<int> idx(n);
    for (int j = 0; j < n; ++j) idx[j] = j;
    Builder B(pb, cen, idx, leaf_max);
    B.nodes.reserve(2 * static_cast<size_t>(n) / std::max(1, leaf_max) + 2);
    const int root = B.build(0, n, 0);
    // flatten: internal nodes in preorder (the root first), leaves as codes
    std::vector<int> pre(B.nodes.size(), -1);
    std::vector<int> order;
    {
        std::vector<int> st{root};
        while (!st.empty()) {
            const int t = st.back();
            st.pop_back();
            if (B.nodes[t].count > 0) continue;
            pre[t] = static_cast<int>(order.size());
            order.push_back(t);
            st.push_back(B.nodes[t].right);
            st.push_back(B.nodes[t].left);
        }
    }
    auto ref = [&](int t) {
        const TNode &x = B.nodes[t];
        if (x.count > 0) return ~((x.first << 3) | (x.count - 1));
        return pre[t];
    };
    hn.clear();
    if (order.empty()) {  // the whole mesh is one leaf: a root whose two children are that leaf
        BNode bn;
        put_child(bn, 0, B.nodes[root].box);
        put_child(bn, 1, B.nodes[root].box);
        bn.ch = make_int4(ref(root), ref(root), 0, 0);
        hn.push_back(bn);
    } else {
        hn.resize(order.size());
        for (size_t i = 0; i < order.size(); ++i) {
            const TNode &x = B.nodes[order[i]];
            BNode bn;
            put_child(bn, 0, B.nodes[x.left].box);
            put_child(bn, 1, B.nodes[x.right].box);
            bn.ch = make_int4(ref(x.left), ref(x.right), 0, 0);
            hn[i] = bn;
        }
    }
    ht.resize(n);
    hs.resize(n);
    for (int j = 0; j < n; ++j) {
        const int li = pm.live[idx[j]];
        const float *a = &pm.v0[3 * li], *b = &pm.e1[3 * li], *c = &pm.e2[3 * li];
        BTri t;
        t.p0 = make_float4(a[0], a[1], a[2], 0.f);
        std::memcpy(&t.p0.w, &li, 4);
        t.p1 = make_float4(b[0], b[1], b[2], 0.0f);
        t.p2 = make_float4(c[0], c[1], c[2], 0.0f);
        ht[j] = t;
        hs[j] = make_float4(pm.n[3 * li], pm.n[3 * li + 1], pm.n[3 * li + 2], 0.0f);
    }
    depth = std::max(1, B.depth);
    return SBR_OK;
}

int validate_layout(const std::vector<BNode> &hn, int n, int leaf_max, int depth, const std::vector<BTri> *tris,
                    int64_t n_ids, const SceneScale *scale)
{
    // every reference in range, every leaf slot covered exactly once, child
    // boxes inside their parent's box, the stack bound respected; with the
    // triangles: every input id in exactly one slot and every triangle's box
    // (the hit rule's box widened by the guard) inside the box its leaf is
    // reached through
    const int nn = static_cast<int>(hn.size());
    std::vector<uint8_t> covered(n, 0);
    std::vector<std::pair<int, int>> st{{0, 0}};
    std::vector<uint8_t> seen(nn, 0);
    int maxd = 0;
    const bool single = nn == 1 && hn[0].ch.x == hn[0].ch.y && hn[0].ch.x < 0;
    while (!st.empty()) {
        const int t = st.back().first, d = st.back().second;
        st.pop_back();
        if (t < 0 || t >= nn || seen[t]) return fail(SBR_ERR_INVALID_MESH, "BVH layout: bad node reference");
        seen[t] = 1;
        maxd = std::max(maxd, d + 1);
        const int refs[2] = {hn[t].ch.x, hn[t].ch.y};
        const float *pf = reinterpret_cast<const float *>(&hn[t]);
        for (int s = 0; s < (single ? 1 : 2); ++s) {
            const int c = refs[s];
            if (c >= 0) {
                if (c <= t) return fail(SBR_ERR_INVALID_MESH, "BVH layout: child before parent");
                const float *cf = reinterpret_cast<const float *>(&hn[c]);
                for (int k = 0; k < 3; ++k)
                    for (int cs = 0; cs < 2; ++cs)
                        if (cf[6 * cs + k] < pf[6 * s + k] || cf[6 * cs + 3 + k] > pf[6 * s + 3 + k])
                            return fail(SBR_ERR_INVALID_MESH, "BVH layout: child box outside its parent");
                st.push_back({c, d + 1});
            } else {
                const int code = ~c, first = code >> 3, cnt = (code & 7) + 1;
                if (cnt > leaf_max || first < 0 || first + cnt > n)
                    return fail(SBR_ERR_INVALID_MESH, "BVH layout: bad leaf");
                for (int q = first; q < first + cnt; ++q) {
                    if (covered[q]) return fail(SBR_ERR_INVALID_MESH, "BVH layout: slot in two leaves");
                    covered[q] = 1;
                    if (!tris) continue;
                    const BTri &tr = (*tris)[q];
                    const float v0[3] = {tr.p0.x, tr.p0.y, tr.p0.z}, e1[3] = {tr.p1.x, tr.p1.y, tr.p1.z},
                                e2[3] = {tr.p2.x, tr.p2.y, tr.p2.z};
                    for (int k = 0; k < 3; ++k) {
                        float lo, hi;
                        spec_box_axis(v0[k], e1[k], e2[k], scale->pbox, lo, hi);
                        if (!(lo - scale->guard >= pf[6 * s + k] && hi + scale->guard <= pf[6 * s + 3 + k]))
                            return fail(SBR_ERR_INVALID_MESH, "BVH layout: triangle box outside its leaf box");
                    }
                }
            }
        }
    }
    for (int q = 0; q < n; ++q)
        if (!covered[q]) return fail(SBR_ERR_INVALID_MESH, "BVH layout: slot in no leaf");
    for (int t = 0; t < nn; ++t)
        if (!seen[t]) return fail(SBR_ERR_INVALID_MESH, "BVH layout: unreachable node");
    if (maxd > depth + 1) return fail(SBR_ERR_INVALID_MESH, "BVH layout: depth bound");
    if (tris) {
        std::vector<uint8_t> used(n_ids, 0);
        for (int q = 0; q < n; ++q) {
            int32_t id;
            std::memcpy(&id, &(*tris)[q].p0.w, 4);
            if (id < 0 || id >= n_ids || used[id]) return fail(SBR_ERR_INVALID_MESH, "BVH layout: bad triangle id");
            used[id] = 1;
        }
    }
    return SBR_OK;
}

void layout_quality(const std::vector<BNode> &hn, sbr_bvh_quality &q)
{
    // surface-area estimates for lines that meet the root box: a node is
    // visited (both child boxes tested) with probability area(node)/area(root),
    // a leaf's triangles are tested with probability area(leaf)/area(root)
    auto area = [](const float *b) {
        const double dx = double(b[3]) - b[0], dy = double(b[4]) - b[1], dz = double(b[5]) - b[2];
        return dx * dy + dy * dz + dz * dx;
    };
    q = sbr_bvh_quality{};
    if (hn.empty()) return;
    const float *r = reinterpret_cast<const float *>(&hn[0]);
    const float root[6] = {std::min(r[0], r[6]), std::min(r[1], r[7]), std::min(r[2], r[8]),
                           std::max(r[3], r[9]), std::max(r[4], r[10]), std::max(r[5], r[11])};
    const double a0 = std::max(area(root), 1e-300);
    const bool single = hn.size() == 1 && hn[0].ch.x == hn[0].ch.y && hn[0].ch.x < 0;
    std::vector<std::pair<int, int>> st{{0, 0}};
    std::vector<double> anode(hn.size(), 0.0);
    anode[0] = 1.0;
    while (!st.empty()) {
        const int t = st.back().first, d = st.back().second;
        st.pop_back();
        q.node_visits += anode[t];
        q.max_depth = std::max(q.max_depth, d + 1);
        const float *pf = reinterpret_cast<const float *>(&hn[t]);
        const int refs[2] = {hn[t].ch.x, hn[t].ch.y};
        for (int s = 0; s < (single ? 1 : 2); ++s) {
            const double ac = area(pf + 6 * s) / a0;
            if (refs[s] >= 0) {
                anode[refs[s]] = ac;
                st.push_back({refs[s], d + 1});
            } else {
                const int cnt = ((~refs[s]) & 7) + 1;
                q.tri_tests += ac * cnt;
                q.leaves += 1;
                q.leaf_tris += cnt;
            }
        }
    }
}

int build_sah(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh)
{
    if (leaf_max < 1 || leaf_max > 4) return fail(SBR_ERR_INVALID_ARG, "leaf size must be in [1, 4]");
    const int64_t nt = bvh->n_tris;
    const int n = static_cast<int>(pm.live.size());
    int rc;
    std::vector<float4> nid(nt);
    for (int64_t j = 0; j < nt; ++j) nid[j] = make_float4(pm.n[3 * j], pm.n[3 * j + 1], pm.n[3 * j + 2], 0.f);
    if ((rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nrm_id), sizeof(float4) * nt))) return rc;
    bvh->n_live = n;
    if (n == 0) {
        bvh->n_nodes = 0;
        bvh->depth = 0;
        return upload_async(ctx, {{bvh->nrm_id, nid.data(), sizeof(float4) * nt}});
    }
    std::vector<BNode> hn;
    std::vector<BTri> ht;
    std::vector<float4> hs;
    int depth = 0;
    if ((rc = sah_layout(pm, leaf_max, hn, ht, hs, depth)) || (rc = validate_layout(hn, n, leaf_max, depth, nullptr, 0, nullptr))) return rc;
    if ((rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nodes), sizeof(BNode) * hn.size())) ||
        (rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->tris), sizeof(BTri) * n)) ||
        (rc = bvh_alloc(bvh, reinterpret_cast<void **>(&bvh->nrm_slot), sizeof(float4) * n)))
        return rc;
    if ((rc = upload_async(ctx, {{bvh->nrm_id, nid.data(), sizeof(float4) * nt},
                                 {bvh->nodes, hn.data(), sizeof(BNode) * hn.size()},
                                 {bvh->tris, ht.data(), sizeof(BTri) * n},
                                 {bvh->nrm_slot, hs.data(), sizeof(float4) * n}})))
        return rc;
    bvh->n_nodes = static_cast<int64_t>(hn.size());
    bvh->depth = depth;
    return SBR_OK;
}

}  // namespace sbr
