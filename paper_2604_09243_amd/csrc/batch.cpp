// Batched sweeps: many (scene, incidence angle, frequency list) items in one
// persistent trace launch per chunk, and the multi-scene arena they trace.
//
// A batch plans every item once (the ray grid of Eqs. L1-L3 over its own
// scene's bounding box, at its own spacing), groups consecutive items into
// chunks of bounded ray count, and owns every device buffer its launches
// touch.  A run is, per chunk: clear the work counters, one streaming trace
// launch in which waves claim 64-ray tiles of any item of the chunk from the
// per-XCD counters (so items of very different sizes share the machine
// without a tail per item), the PO launch over the chunk's records (one block
// per 4096 records of an item, all frequencies of that item) and the
// finalize launch.  The whole sequence is captured once into a HIP graph on
// a private stream and replayed on the context stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "sbr_internal.hpp"

using namespace sbr;

namespace {

struct DevBufs {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    void release()
    {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
    template <class T>
    int alloc(T **p, size_t n)
    {
        const size_t b = std::max<size_t>(sizeof(T) * n, 256);
        void *q = nullptr;
        if (hipMalloc(&q, b) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SBR_ERR_OOM, "batch: device allocation of " + std::to_string(b) + " bytes failed");
        }
        ptrs.push_back(q);
        bytes += static_cast<int64_t>(b);
        *p = static_cast<T *>(q);
        return SBR_OK;
    }
};

struct EventSet {
    std::vector<hipEvent_t> ev;
    ~EventSet()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    int create(size_t n)
    {
        ev.assign(n, nullptr);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(SBR_ERR_HIP, "batch: hipEventCreate failed");
        return SBR_OK;
    }
};

}  // namespace

struct sbr_batch {
    sbr_ctx *ctx = nullptr;
    int device = 0;  // kept so that destroying the batch never reads the context
    const sbr_bvh *bvh = nullptr;
    std::vector<sbr_batch_item> items;
    std::vector<double> freqs;
    int bmax = 5, mode = SBR_MODE_VECTOR;
    uint32_t flags = 0;
    double eta = 0.1;
    sbr_tune tune{};
    // per item (host)
    std::vector<sbr_angle_plan> hplan;
    std::vector<double> ds;
    std::vector<int64_t> out_base;
    int64_t n_rows = 0, rays = 0, min_rays = 0, max_rays = 0;
    // chunks: items [cstart[c], cstart[c + 1])
    std::vector<int64_t> cstart, c_tiles, c_units, tile_off, c_rays;
    std::vector<int> c_maxnf;
    std::vector<int> c_kinds;  // per chunk: kPoEven | kPoUneven of its items
    std::vector<int64_t> c_mask_bytes, c_mask_units;  // primary-ray mask of each chunk
    int blocks = 0;
    // device
    DevBufs dev;
    AnglePlan *d_plans = nullptr;
    int64_t *d_tile = nullptr;
    PoAngle *d_ang = nullptr;
    double *d_kf = nullptr;
    Records rec{};
    long long *d_part = nullptr;
    uint32_t *d_ctr = nullptr;
    CounterPtrs ctrs{};
    int32_t *d_spill = nullptr;
    uint8_t *d_mask = nullptr;  // NULL with SBR_OPT_NO_MASK
    int32_t *d_live = nullptr;  // live tiles of a chunk (streaming schedule with the mask)
    uint32_t *d_liveblk = nullptr;
    RayQueue qa{}, qb{};
    unsigned long long *h_stat = nullptr;  // pinned [kStatU64]
    // graph
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double *g_A = nullptr, *g_sigma = nullptr;
    bool graph_ready = false;
};

namespace {

struct SceneView {
    int32_t root;
    float eps;
    double diag;
    const double *bbox;
    int64_t n_nodes;
};

SceneView scene_view(const sbr_bvh *b, int s)
{
    if (b->scenes.empty()) return SceneView{0, b->eps, b->diag, b->bbox, b->n_nodes};
    const SceneInfo &si = b->scenes[s];
    return SceneView{si.root, si.eps, si.diag, si.bbox, si.n_nodes};
}

int n_scenes(const sbr_bvh *b) { return b->scenes.empty() ? 1 : static_cast<int>(b->scenes.size()); }

void drop_graph(sbr_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ready = false;
}

// Chunks and device buffers for the batch's current tune.
int plan_batch(sbr_batch *b)
{
    drop_graph(b);
    SBR_HIP(hipSetDevice(b->ctx->device));
    SBR_HIP(hipStreamSynchronize(b->ctx->stream));  // an earlier run may still use the buffers
    b->dev.release();
    const sbr_bvh *bv = b->bvh;
    const int64_t ni = static_cast<int64_t>(b->items.size());
    const int tw = b->tune.tile_w;
    const int64_t cap = int64_t(1) << b->tune.chunk_log2;
    std::vector<AnglePlan> plans(ni);
    std::vector<PoAngle> ang(ni);
    std::vector<double> kf(b->freqs.size());
    for (size_t f = 0; f < kf.size(); ++f) kf[f] = 2.0 * kPi * b->freqs[f] / kC0;
    for (int64_t i = 0; i < ni; ++i) {
        const sbr_batch_item &it = b->items[i];
        const sbr_angle_plan &ap = b->hplan[i];
        const SceneView sv = scene_view(bv, it.scene);
        AnglePlan &p = plans[i];
        fill_plan(ap, b->ds[i], tw, p);
        int rc;
        if ((rc = scene_plan(p, sv.root, sv.eps, sv.bbox, sv.diag, sv.n_nodes))) return rc;
        PoAngle &q = ang[i];
        for (int k = 0; k < 3; ++k) {
            q.basis[k] = ap.k_hat[k];
            q.basis[3 + k] = ap.theta_hat[k];
            q.basis[6 + k] = ap.phi_hat[k];
        }
        q.dA = b->ds[i] * b->ds[i];
        q.rec_cnt = ap.nu * ap.nv;
        q.out_base = b->out_base[i];
        q.kf_off = static_cast<int32_t>(it.freq_offset);
        q.n_f = it.n_freq;
        q.dk = uniform_step(kf.data() + it.freq_offset, it.n_freq);
    }
    b->cstart.clear();
    b->c_tiles.clear();
    b->c_units.clear();
    b->c_maxnf.clear();
    b->c_kinds.clear();
    b->c_rays.clear();
    b->tile_off.clear();
    b->c_mask_bytes.clear();
    b->c_mask_units.clear();
    int64_t max_rays = 0, max_rows = 0, tile_words = 0, max_mask = 4, max_tiles = 1;
    for (int64_t a = 0; a < ni;) {
        b->cstart.push_back(a);
        b->tile_off.push_back(tile_words);
        int64_t rays = 0, tiles = 0, units = 0, rows = 0, e = a;
        int mnf = 1, kinds = 0;
        while (e < ni) {
            const int64_t r = ang[e].rec_cnt;
            if (e > a && rays + r > cap) break;
            plans[e].tile_base = tiles;
            plans[e].rec_base = rays;
            ang[e].rec_base = rays;
            ang[e].unit_base = units;
            ang[e].part_base = rows;
            tiles += int64_t(plans[e].tu) * plans[e].tv;
            rays += r;
            units += po_units(r);
            rows += po_units(r) * ang[e].n_f;
            mnf = std::max(mnf, ang[e].n_f);
            kinds |= po_kind(ang[e].dk);
            ++e;
        }
        b->c_tiles.push_back(tiles);
        b->c_rays.push_back(rays);
        b->c_units.push_back(units);
        b->c_maxnf.push_back(mnf);
        b->c_kinds.push_back(kinds);
        int64_t mb = 0, mu = 0;
        mask_layout(plans.data(), a, e, mb, mu);
        b->c_mask_bytes.push_back(mb);
        b->c_mask_units.push_back(mu);
        max_mask = std::max(max_mask, mb);
        tile_words += (e - a) + 1;
        max_rays = std::max(max_rays, rays);
        max_rows = std::max(max_rows, rows);
        max_tiles = std::max(max_tiles, tiles);
        a = e;
    }
    b->cstart.push_back(ni);
    const int n_chunks = static_cast<int>(b->cstart.size()) - 1;
    if (b->c_units.size() && *std::max_element(b->c_units.begin(), b->c_units.end()) > 2147483647LL)
        return fail(SBR_ERR_OVERFLOW, "sbr_batch: too many PO blocks in one chunk");
    std::vector<int64_t> tb(tile_words);
    for (int c = 0; c < n_chunks; ++c) {
        int64_t w = b->tile_off[c];
        for (int64_t a = b->cstart[c]; a < b->cstart[c + 1]; ++a) tb[w++] = plans[a].tile_base;
        tb[w] = b->c_tiles[c];
    }
    b->blocks = trace_persistent_blocks(b->ctx, b->tune.blocks_per_cu);
    int rc;
    Rec *recs;
    uint32_t *held;
    if ((rc = b->dev.alloc(&b->d_plans, ni)) || (rc = b->dev.alloc(&b->d_tile, tile_words)) ||
        (rc = b->dev.alloc(&b->d_ang, ni)) || (rc = b->dev.alloc(&b->d_kf, b->freqs.size())) ||
        (rc = b->dev.alloc(&recs, max_rays)) ||
        (rc = b->dev.alloc(&held, static_cast<size_t>(held_words(max_rays)))) ||
        (rc = b->dev.alloc(&b->d_part, 8 * static_cast<size_t>(max_rows))) ||
        (rc = b->dev.alloc(&b->d_ctr, kCounterBytes / 4)) ||
        (rc = b->dev.alloc(&b->d_spill, spill_words(bv, b->blocks))))
        return rc;
    b->d_mask = nullptr;
    b->d_live = nullptr;
    b->d_liveblk = nullptr;
    if (!(b->flags & SBR_OPT_NO_MASK)) {
        if ((rc = b->dev.alloc(&b->d_mask, static_cast<size_t>((max_mask + 3) & ~int64_t(3))))) return rc;
        // the streaming schedule claims the live tiles of the mask
        if (b->tune.schedule == kScheduleStream &&
            ((rc = b->dev.alloc(&b->d_live, static_cast<size_t>(max_tiles))) ||
             (rc = b->dev.alloc(&b->d_liveblk, static_cast<size_t>(live_blocks(max_tiles) + 1)))))
            return rc;
    }
    b->rec = Records{recs, reinterpret_cast<uint8_t *>(held)};
    char *cb = reinterpret_cast<char *>(b->d_ctr);
    b->ctrs.stat = reinterpret_cast<unsigned long long *>(cb);
    b->ctrs.q_cnt = reinterpret_cast<uint32_t *>(cb + kStatBytes);
    b->ctrs.claim = b->ctrs.q_cnt + static_cast<size_t>(kLineU32) * kQcnt;
    if (b->tune.schedule == kScheduleWavefront) {
        RayQueue *qs[2] = {&b->qa, &b->qb};
        for (RayQueue *q : qs)
            if ((rc = b->dev.alloc(&q->s0, max_rays)) || (rc = b->dev.alloc(&q->s1, max_rays)) ||
                (rc = b->dev.alloc(&q->s2, max_rays)) || (rc = b->dev.alloc(&q->s3, max_rays)) ||
                (rc = b->dev.alloc(&q->s4, max_rays)) || (rc = b->dev.alloc(&q->s5, max_rays)))
                return rc;
    } else {
        b->qa = RayQueue{};
        b->qb = RayQueue{};
    }
    SBR_HIP(hipMemcpy(b->d_plans, plans.data(), sizeof(AnglePlan) * ni, hipMemcpyHostToDevice));
    SBR_HIP(hipMemcpy(b->d_tile, tb.data(), 8 * tile_words, hipMemcpyHostToDevice));
    SBR_HIP(hipMemcpy(b->d_ang, ang.data(), sizeof(PoAngle) * ni, hipMemcpyHostToDevice));
    SBR_HIP(hipMemcpy(b->d_kf, kf.data(), 8 * kf.size(), hipMemcpyHostToDevice));
    return SBR_OK;
}

// The launches of one run.  ev (nullable): 3 events per chunk (before the
// trace, after the trace, after the PO stage).
int enqueue(sbr_batch *b, hipStream_t s, double *A, double *sigma, std::vector<hipEvent_t> *ev)
{
    int rc;
    const int64_t ctr_words = static_cast<int64_t>(kCounterBytes / 4);
    const int64_t stat_words = static_cast<int64_t>(kStatBytes / 4);
    if ((rc = launch_zero_u32(s, b->d_ctr, ctr_words))) return rc;
    const int n_chunks = static_cast<int>(b->cstart.size()) - 1;
    for (int c = 0; c < n_chunks; ++c) {
        const int64_t a0 = b->cstart[c], a1 = b->cstart[c + 1];
        // the statistics accumulate over chunks; queue and claim counters restart
        if (c > 0 && (rc = launch_zero_u32(s, b->d_ctr + stat_words, ctr_words - stat_words))) return rc;
        if (ev) SBR_HIP(hipEventRecord((*ev)[3 * c], s));
        // the chunk's record slots start empty
        if ((rc = launch_zero_u32(s, reinterpret_cast<uint32_t *>(b->rec.held), held_words(b->c_rays[c])))) return rc;
        TraceArgs ta{};
        ta.bvh = b->bvh;
        ta.bmax = b->bmax;
        ta.flags = b->flags;
        ta.schedule = b->tune.schedule;
        ta.tile_shift = log2i(b->tune.tile_w);
        ta.claim_tiles = b->tune.claim_tiles ? b->tune.claim_tiles : auto_claim_tiles(b->bvh);
        ta.refill_min = b->tune.refill_min;
        ta.blocks = b->blocks;
        ta.plans = b->d_plans + a0;
        ta.tile_base = b->d_tile + b->tile_off[c];
        ta.n_angles = static_cast<int>(a1 - a0);
        ta.n_tiles = b->c_tiles[c];
        ta.rec = b->rec;
        ta.ctrs = b->ctrs;
        ta.spill = b->d_spill;
        if (b->d_mask) {
            ta.mask = b->d_mask;
            if ((rc = launch_mask(s, b->bvh->nodes, ta.plans, ta.n_angles, b->c_mask_units[c], b->d_mask,
                                  b->c_mask_bytes[c])))
                return rc;
            if (b->d_live) {
                if ((rc = launch_live(s, ta, b->d_live, b->d_liveblk))) return rc;
                ta.live = b->d_live;
                ta.live_count = b->d_liveblk + live_blocks(ta.n_tiles);
            }
        }
        if ((rc = run_trace(s, ta, b->qa, b->qb, nullptr))) return rc;
        if (ev) SBR_HIP(hipEventRecord((*ev)[3 * c + 1], s));
        PoArgs pa{};
        pa.bvh = b->bvh;
        pa.rec = b->rec;
        pa.rec_slots = 1;
        pa.ang = b->d_ang + a0;
        pa.n_angles = static_cast<int>(a1 - a0);
        pa.n_units = b->c_units[c];
        pa.max_nf = b->c_maxnf[c];
        pa.kinds = b->c_kinds[c];
        pa.mode = b->mode;
        pa.kf = b->d_kf;
        pa.partial = b->d_part;
        if ((rc = launch_po(s, pa)) || (rc = launch_po_finalize(s, pa, A, sigma))) return rc;
        if (ev) SBR_HIP(hipEventRecord((*ev)[3 * c + 2], s));
    }
    return SBR_OK;
}

int capture(sbr_batch *b, double *A, double *sigma)
{
    drop_graph(b);
    if (!b->cap) SBR_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    SBR_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(b, b->cap, A, sigma, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != SBR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return fail(SBR_ERR_HIP, std::string("sbr_batch_run: graph capture failed: ") + hipGetErrorString(e));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SBR_ERR_HIP, std::string("sbr_batch_run: graph instantiation failed: ") + hipGetErrorString(ei));
    }
    b->graph = g;
    b->exec = x;
    b->g_A = A;
    b->g_sigma = sigma;
    b->graph_ready = true;
    return SBR_OK;
}

void destroy_batch(sbr_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();  // the batch's last run may still be in flight
    drop_graph(b);
    b->dev.release();
    if (b->h_stat) (void)hipHostFree(b->h_stat);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

}  // namespace

// ---------------------------------------------------------------- scene sets
extern "C" int sbr_pack_scenes(sbr_ctx *ctx, const sbr_bvh *const *bvhs, int n_bvhs, sbr_bvh **out)
{
    if (!ctx || !bvhs || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_pack_scenes: NULL argument");
    *out = nullptr;
    if (n_bvhs < 1 || n_bvhs > 65536) return fail(SBR_ERR_INVALID_ARG, "sbr_pack_scenes: n_bvhs must be in [1, 65536]");
    int64_t tn = 0, tl = 0, tt = 0;
    for (int s = 0; s < n_bvhs; ++s) {
        const sbr_bvh *b = bvhs[s];
        if (!b) return fail(SBR_ERR_INVALID_ARG, "sbr_pack_scenes: NULL BVH " + std::to_string(s));
        if (b->device != ctx->device) return fail(SBR_ERR_INVALID_ARG, "sbr_pack_scenes: BVH on another device");
        if (!b->scenes.empty()) return fail(SBR_ERR_INVALID_ARG, "sbr_pack_scenes: a BVH is itself a scene set");
        if (b->n_live == 0 || b->n_nodes == 0)
            return fail(SBR_ERR_INVALID_ARG, "sbr_pack_scenes: scene " + std::to_string(s) + " has no triangle");
        tn += b->n_nodes;
        tl += b->n_live;
        tt += b->n_tris;
    }
    if (tt > (int64_t(1) << 28) || tn > 2147483647LL || tl * 8 > 2147483647LL)
        return fail(SBR_ERR_OVERFLOW, "sbr_pack_scenes: more than 2^28 triangles in total");
    SBR_HIP(hipSetDevice(ctx->device));
    sbr_bvh *set = new (std::nothrow) sbr_bvh();
    if (!set) return fail(SBR_ERR_OOM, "sbr_pack_scenes: out of host memory");
    set->device = ctx->device;
    auto dalloc = [&](void **p, size_t bytes) -> int { return bvh_alloc(set, p, bytes); };
    int rc;
    if ((rc = dalloc(reinterpret_cast<void **>(&set->nodes), sizeof(BNode) * tn)) ||
        (rc = dalloc(reinterpret_cast<void **>(&set->tris), sizeof(BTri) * tl)) ||
        (rc = dalloc(reinterpret_cast<void **>(&set->nrm_slot), sizeof(float4) * tl)) ||
        (rc = dalloc(reinterpret_cast<void **>(&set->nrm_id), sizeof(float4) * tt))) {
        sbr_free_bvh(set);
        return rc;
    }
    hipStream_t st = ctx->stream;
    int64_t no = 0, so = 0, io = 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    set->scenes.resize(n_bvhs);
    set->host_normals.reserve(3 * tt);
    for (int s = 0; s < n_bvhs; ++s) {
        const sbr_bvh *b = bvhs[s];
        rc = launch_relocate(st, b->nodes, b->n_nodes, set->nodes + no, static_cast<int32_t>(no), b->tris, b->n_live,
                             set->tris + so, static_cast<int32_t>(so), static_cast<int32_t>(io));
        if (rc == SBR_OK &&
            (hipMemcpyAsync(set->nrm_slot + so, b->nrm_slot, sizeof(float4) * b->n_live, hipMemcpyDeviceToDevice, st) !=
                 hipSuccess ||
             hipMemcpyAsync(set->nrm_id + io, b->nrm_id, sizeof(float4) * b->n_tris, hipMemcpyDeviceToDevice, st) !=
                 hipSuccess))
            rc = fail(SBR_ERR_HIP, "sbr_pack_scenes: device copy failed");
        if (rc) {
            (void)hipStreamSynchronize(st);
            sbr_free_bvh(set);
            return rc;
        }
        SceneInfo &si = set->scenes[s];
        si.root = static_cast<int32_t>(no);
        si.slot_base = static_cast<int32_t>(so);
        si.id_base = static_cast<int32_t>(io);
        si.depth = b->depth;
        si.n_tris = b->n_tris;
        si.n_live = b->n_live;
        si.n_nodes = b->n_nodes;
        si.eps = b->eps;
        si.diag = b->diag;
        std::memcpy(si.bbox, b->bbox, sizeof(si.bbox));
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b->bbox[k]);
            hi[k] = std::max(hi[k], b->bbox[3 + k]);
        }
        set->host_normals.insert(set->host_normals.end(), b->host_normals.begin(), b->host_normals.end());
        set->depth = std::max(set->depth, b->depth);
        set->leaf_size = std::max(set->leaf_size, b->leaf_size);
        set->eps = std::max(set->eps, b->eps);
        no += b->n_nodes;
        so += b->n_live;
        io += b->n_tris;
    }
    set->n_tris = tt;
    set->n_live = tl;
    set->n_nodes = tn;
    for (int k = 0; k < 3; ++k) {
        set->bbox[k] = lo[k];
        set->bbox[3 + k] = hi[k];
    }
    set->diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                          (hi[2] - lo[2]) * (hi[2] - lo[2]));
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        sbr_free_bvh(set);
        return fail(SBR_ERR_HIP, std::string("sbr_pack_scenes: ") + hipGetErrorString(e));
    }
    *out = set;
    return SBR_OK;
}

// ---------------------------------------------------------------- batches
extern "C" int sbr_batch_create(sbr_ctx *ctx, const sbr_bvh *scenes, const sbr_batch_desc *d, sbr_batch **out)
{
    if (!ctx || !scenes || !d || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: NULL argument");
    *out = nullptr;
    if (d->struct_size < sizeof(sbr_batch_desc))
        return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: desc->struct_size too small");
    if (!d->items || d->n_items < 1 || d->n_items > (int64_t(1) << 24))
        return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: n_items must be in [1, 2^24]");
    if (!d->freqs_hz || d->n_freqs_total < 1 || d->n_freqs_total > 2147483647LL)
        return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: empty frequency array");
    if (d->max_bounces < 1 || d->max_bounces > SBR_MAX_BOUNCES)
        return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: max_bounces must be in [1, " + std::to_string(SBR_MAX_BOUNCES) + "]");
    if (d->mode != SBR_MODE_VECTOR && d->mode != SBR_MODE_PAPER)
        return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: unknown mode");
    if (scenes->device != ctx->device) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: scenes on another device");
    if (scenes->n_live == 0) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: the scenes hold no triangle");
    for (int64_t f = 0; f < d->n_freqs_total; ++f)
        if (!(d->freqs_hz[f] > 0.0) || !std::isfinite(d->freqs_hz[f]))
            return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: frequencies must be positive and finite");
    sbr_tune tune = default_tune();  // chunk_log2 0: automatic
    if (d->tune) {
        if (d->tune->struct_size < sizeof(sbr_tune))
            return fail(SBR_ERR_INVALID_ARG, "sbr_batch_create: tune->struct_size too small");
        tune = *d->tune;
    }
    if (d->flags & (SBR_OPT_FP32_PATH | SBR_OPT_FP64_TRAVERSE))
        return fail(SBR_ERR_UNSUPPORTED,
                    "sbr_batch_create: SBR_OPT_FP32_PATH and SBR_OPT_FP64_TRAVERSE are study options of sweeps and traces");
    if (d->flags & SBR_OPT_WAVEFRONT) tune.schedule = kScheduleWavefront;
    if (tune.chunk_log2 == 0) {
        SBR_HIP(hipSetDevice(ctx->device));
        tune.chunk_log2 = auto_chunk_log2(0);
    }
    int rc = normalize_tune(tune);
    if (rc) return rc;
    const int ns = n_scenes(scenes);
    const double eta = d->eta < 0.0 ? 0.1 : d->eta;
    sbr_batch *b = new (std::nothrow) sbr_batch();
    if (!b) return fail(SBR_ERR_OOM, "sbr_batch_create: out of host memory");
    b->ctx = ctx;
    b->device = ctx->device;
    b->bvh = scenes;
    b->items.assign(d->items, d->items + d->n_items);
    b->freqs.assign(d->freqs_hz, d->freqs_hz + d->n_freqs_total);
    b->bmax = d->max_bounces;
    b->mode = d->mode;
    b->flags = d->flags;
    b->eta = eta;
    b->tune = tune;
    const int64_t ni = d->n_items;
    b->hplan.resize(ni);
    b->ds.resize(ni);
    b->out_base.resize(ni);
    b->min_rays = INT64_MAX;
    for (int64_t i = 0; i < ni; ++i) {
        const sbr_batch_item &it = b->items[i];
        std::string where = "sbr_batch_create: item " + std::to_string(i) + ": ";
        if (it.scene < 0 || it.scene >= ns) rc = fail(SBR_ERR_INVALID_ARG, where + "scene index out of range");
        else if (it.n_freq < 1 || it.n_freq > 4096) rc = fail(SBR_ERR_INVALID_ARG, where + "n_freq must be in [1, 4096]");
        else if (it.freq_offset < 0 || it.freq_offset + it.n_freq > d->n_freqs_total)
            rc = fail(SBR_ERR_INVALID_ARG, where + "frequencies outside freqs_hz");
        if (rc) break;
        double fmax = 0.0;
        for (int f = 0; f < it.n_freq; ++f) fmax = std::max(fmax, d->freqs_hz[it.freq_offset + f]);
        double ds = it.ds;
        if (!(ds > 0.0)) {
            if (!(d->samples_per_lambda > 0.0)) {
                rc = fail(SBR_ERR_INVALID_ARG, where + "give ds or samples_per_lambda");
                break;
            }
            ds = kC0 / fmax / d->samples_per_lambda;
        }
        // sampling rule of Sec. 4: ds <= lambda / 5 at the item's highest frequency
        if (ds > (kC0 / fmax / 5.0) * (1.0 + 1e-12) && !(d->flags & SBR_OPT_ALLOW_UNDERSAMPLING)) {
            rc = fail(SBR_ERR_SAMPLING, where + "ray spacing exceeds lambda/5 at its highest frequency");
            break;
        }
        const SceneView sv = scene_view(scenes, it.scene);
        if ((rc = plan_angle(sv.bbox, it.theta_deg, it.phi_deg, ds, eta, b->hplan[i]))) break;
        const int64_t r = b->hplan[i].nu * b->hplan[i].nv;
        if (r > (int64_t(1) << 31) - 1) {
            rc = fail(SBR_ERR_OVERFLOW, where + "too many rays");
            break;
        }
        b->ds[i] = ds;
        b->out_base[i] = b->n_rows;
        b->n_rows += it.n_freq;
        b->rays += r;
        b->min_rays = std::min(b->min_rays, r);
        b->max_rays = std::max(b->max_rays, r);
    }
    if (rc == SBR_OK && hipHostMalloc(reinterpret_cast<void **>(&b->h_stat), 8 * kStatU64, hipHostMallocDefault) !=
                            hipSuccess) {
        (void)hipGetLastError();
        b->h_stat = nullptr;
        rc = fail(SBR_ERR_OOM, "sbr_batch_create: pinned host allocation failed");
    }
    if (rc == SBR_OK) rc = plan_batch(b);
    if (rc) {
        destroy_batch(b);
        return rc;
    }
    *out = b;
    return SBR_OK;
}

extern "C" int sbr_batch_get_info(const sbr_batch *b, sbr_batch_info *out)
{
    if (!b || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_get_info: NULL argument");
    out->n_items = static_cast<int64_t>(b->items.size());
    out->n_rows = b->n_rows;
    out->rays = b->rays;
    out->min_item_rays = b->min_rays;
    out->max_item_rays = b->max_rays;
    out->n_chunks = static_cast<int32_t>(b->cstart.size()) - 1;
    out->graph_ready = b->graph_ready ? 1 : 0;
    out->device_bytes = b->dev.bytes;
    out->tune = b->tune;
    return SBR_OK;
}

extern "C" int sbr_batch_set_tune(sbr_batch *b, const sbr_tune *t)
{
    if (!b || !t) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_set_tune: NULL argument");
    if (t->struct_size < sizeof(sbr_tune)) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_set_tune: struct_size too small");
    sbr_tune n = *t;
    if (b->flags & SBR_OPT_WAVEFRONT) n.schedule = kScheduleWavefront;
    if (n.chunk_log2 == 0) {  // the batch's own record slots count as free: the new plan replaces them
        SBR_HIP(hipSetDevice(b->device));
        int64_t mr = 0;
        for (const int64_t r : b->c_rays) mr = std::max(mr, r);
        n.chunk_log2 = auto_chunk_log2(static_cast<size_t>(mr) * (sizeof(Rec) + 1));
    }
    int rc = normalize_tune(n);
    if (rc) return rc;
    b->tune = n;
    return plan_batch(b);
}

extern "C" int sbr_batch_run(sbr_batch *b, double *A_out, double *sigma_dbsm, sbr_stats *stats)
{
    const auto t_start = std::chrono::steady_clock::now();
    if (!b || !A_out) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_run: NULL argument");
    SBR_HIP(hipSetDevice(b->ctx->device));
    hipStream_t s = b->ctx->stream;
    const bool eager = (b->flags & SBR_OPT_NO_GRAPH) != 0;
    const int n_chunks = static_cast<int>(b->cstart.size()) - 1;
    EventSet es;
    int rc;
    if (eager) {
        if (stats && (rc = es.create(3 * static_cast<size_t>(n_chunks)))) return rc;
        if ((rc = enqueue(b, s, A_out, sigma_dbsm, stats ? &es.ev : nullptr))) return rc;
    } else {
        if (!b->graph_ready || b->g_A != A_out || b->g_sigma != sigma_dbsm) {
            if ((rc = capture(b, A_out, sigma_dbsm))) return rc;
        }
        if (stats) {
            if ((rc = es.create(2))) return rc;
            SBR_HIP(hipEventRecord(es.ev[0], s));
        }
        SBR_HIP(hipGraphLaunch(b->exec, s));
        if (stats) SBR_HIP(hipEventRecord(es.ev[1], s));
    }
    if (stats || (b->flags & SBR_OPT_SYNC)) {
        SBR_HIP(hipMemcpyAsync(b->h_stat, b->ctrs.stat, 8 * kStatU64, hipMemcpyDeviceToHost, s));
        SBR_HIP(hipStreamSynchronize(s));
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->rays = b->rays;
        fill_stats(stats, b->h_stat, b->bmax, b->rays, (b->flags & SBR_OPT_DROP_TRAPPED) != 0,
                   b->tune.schedule == kScheduleStream ? n_chunks : 0);
        stats->angles = static_cast<int64_t>(b->items.size());
        if (eager) {
            for (int c = 0; c < n_chunks; ++c) {
                float t1 = 0, t2 = 0;
                SBR_HIP(hipEventElapsedTime(&t1, es.ev[3 * c], es.ev[3 * c + 1]));
                SBR_HIP(hipEventElapsedTime(&t2, es.ev[3 * c + 1], es.ev[3 * c + 2]));
                stats->ms_trace += t1;
                stats->ms_po += t2;
            }
        } else {
            float t = 0;
            SBR_HIP(hipEventElapsedTime(&t, es.ev[0], es.ev[1]));
            stats->ms_total = t;
        }
        if (eager)
            stats->ms_total =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return SBR_OK;
}

extern "C" int sbr_batch_autotune(sbr_batch *b, sbr_tune *out)
{
    if (!b || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_batch_autotune: NULL argument");
    sbr_ctx *ctx = b->ctx;
    char key[256];
    std::snprintf(key, sizeof(key), "batch|%s|r%d|i%d|t%d|b%d", ctx->prop.gcnArchName,
                  size_bucket(static_cast<double>(b->rays)), size_bucket(static_cast<double>(b->items.size())),
                  size_bucket(static_cast<double>(b->bvh->n_live)), b->bmax);
    sbr_tune t;
    int rc;
    if (tune_lookup(ctx, key, &t)) {
        if ((rc = sbr_batch_set_tune(b, &t))) return rc;
        *out = b->tune;
        return SBR_OK;
    }
    // sample: every 8th item (all of them for small batches)
    const int64_t ni = static_cast<int64_t>(b->items.size());
    const int64_t stride = ni >= 16 ? 8 : 1;
    std::vector<sbr_batch_item> sub;
    for (int64_t i = 0; i < ni; i += stride) {
        sbr_batch_item it = b->items[i];
        it.ds = b->ds[i];
        sub.push_back(it);
    }
    sbr_batch_desc d{};
    d.struct_size = sizeof(d);
    d.items = sub.data();
    d.n_items = static_cast<int64_t>(sub.size());
    d.freqs_hz = b->freqs.data();
    d.n_freqs_total = static_cast<int64_t>(b->freqs.size());
    d.max_bounces = b->bmax;
    d.mode = b->mode;
    d.flags = b->flags & ~static_cast<uint32_t>(SBR_OPT_NO_GRAPH | SBR_OPT_SYNC);
    d.samples_per_lambda = 0.0;
    d.eta = b->eta;
    d.tune = &b->tune;
    sbr_batch *sb = nullptr;
    if ((rc = sbr_batch_create(ctx, b->bvh, &d, &sb))) return rc;
    double *dA = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&dA), 64 * static_cast<size_t>(sb->n_rows)) != hipSuccess) {
        (void)hipGetLastError();
        destroy_batch(sb);
        return fail(SBR_ERR_OOM, "sbr_batch_autotune: device allocation failed");
    }
    auto eval = [&](const sbr_tune &c, double *ms) -> int {
        int r = sbr_batch_set_tune(sb, &c);
        if (r) return r;
        double best = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            sbr_stats st;
            if ((r = sbr_batch_run(sb, dA, nullptr, &st))) return r;
            if (rep > 0) best = std::min(best, st.ms_total);  // the first run captures and warms caches
        }
        *ms = best;
        return SBR_OK;
    };
    sbr_tune cur = b->tune;
    double cur_ms = 0;
    rc = eval(cur, &cur_ms);
    const int refills[] = {1, 16, 32, 64};
    const int tiles[] = {4, 8, 16, 32};
    const int claims[] = {1, 2, 4, 8};
    const int blocks[] = {0, 2};
    const int chunks[] = {22, 24, 26};
    for (int pass = 0; pass < 5 && rc == SBR_OK; ++pass) {
        const int *vals = pass == 0 ? refills : pass == 1 ? tiles : pass == 2 ? claims : pass == 3 ? blocks : chunks;
        const int nv = pass == 3 ? 2 : pass == 4 ? 3 : 4;
        for (int v = 0; v < nv && rc == SBR_OK; ++v) {
            sbr_tune c = cur;
            int &field = pass == 0   ? c.refill_min
                         : pass == 1 ? c.tile_w
                         : pass == 2 ? c.claim_tiles
                         : pass == 3 ? c.blocks_per_cu
                                     : c.chunk_log2;
            if (field == vals[v]) continue;
            field = vals[v];
            double ms = 0;
            if ((rc = eval(c, &ms))) break;
            if (ms < cur_ms) {
                cur_ms = ms;
                cur = c;
            }
        }
    }
    (void)hipFree(dA);
    destroy_batch(sb);
    if (rc) return rc;
    tune_store(ctx, key, cur);
    if ((rc = sbr_batch_set_tune(b, &cur))) return rc;
    *out = b->tune;
    return SBR_OK;
}

extern "C" void sbr_batch_destroy(sbr_batch *b) { destroy_batch(b); }
