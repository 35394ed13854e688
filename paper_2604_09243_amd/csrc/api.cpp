// C ABI of the SBR library: context, workspace, argument checking and the
// orchestration of the kernels of each entry point.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "sbr_internal.hpp"

namespace sbr {

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int status, const std::string &msg)
{
    g_err = msg;
    return status;
}

// ---------------------------------------------------------------- BVH blocks
namespace {
struct BlockCache {
    std::mutex m;
    std::map<int, std::multimap<size_t, void *>> free;  // device -> (size class, block)
    size_t held = 0;
};
BlockCache &block_cache()
{
    static BlockCache *c = new BlockCache();  // lives to the end of the process
    return *c;
}
constexpr size_t kBlockCacheMax = size_t(1) << 30;
size_t size_class(size_t bytes)
{
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    return c;
}
}  // namespace

int device_block_get(int device, size_t bytes, void **p, size_t *cap)
{
    const size_t c = size_class(bytes);
    *cap = c;
    {
        BlockCache &bc = block_cache();
        std::lock_guard<std::mutex> g(bc.m);
        auto &fl = bc.free[device];
        auto it = fl.find(c);
        if (it != fl.end()) {
            *p = it->second;
            fl.erase(it);
            bc.held -= c;
            return SBR_OK;
        }
    }
    if (hipMalloc(p, c) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(SBR_ERR_OOM, "device allocation of " + std::to_string(c) + " bytes failed");
    }
    return SBR_OK;
}

void device_block_put(int device, void *p, size_t cap)
{
    if (!p) return;
    BlockCache &bc = block_cache();
    std::lock_guard<std::mutex> g(bc.m);
    if (bc.held + cap <= kBlockCacheMax) {
        bc.free[device].emplace(cap, p);
        bc.held += cap;
    } else {
        (void)hipFree(p);
    }
}

int bvh_alloc(sbr_bvh *bvh, void **p, size_t bytes)
{
    size_t c = 0;
    const int rc = device_block_get(bvh->device, bytes, p, &c);
    if (rc) return rc;
    bvh->blocks.emplace_back(*p, c);
    bvh->device_bytes += static_cast<int64_t>(c);
    return SBR_OK;
}

int upload_async(sbr_ctx *ctx, const std::vector<Upload> &ups)
{
    size_t total = 0;
    for (const auto &u : ups) total += (u.bytes + 255) & ~size_t(255);
    if (total == 0) return SBR_OK;
    SBR_HIP(hipStreamSynchronize(ctx->stream));  // the staging buffer may still feed an earlier copy
    void *pin = nullptr;
    int rc = ctx->ws->get_pinned(total, &pin);
    if (rc) return rc;
    char *q = static_cast<char *>(pin);
    for (const auto &u : ups) {
        std::memcpy(q, u.src, u.bytes);
        SBR_HIP(hipMemcpyAsync(u.dst, q, u.bytes, hipMemcpyHostToDevice, ctx->stream));
        q += (u.bytes + 255) & ~size_t(255);
    }
    return SBR_OK;
}

// ---------------------------------------------------------------- workspace
Workspace::~Workspace()
{
    for (auto &b : bufs)
        if (b.p) (void)hipFree(b.p);
    if (pinned) (void)hipHostFree(pinned);
}

int Workspace::get(int i, size_t bytes, void **out)
{
    if (static_cast<int>(bufs.size()) <= i) bufs.resize(i + 1);
    Buf &b = bufs[i];
    if (b.bytes < bytes) {
        if (b.p) {
            (void)hipFree(b.p);
            b.p = nullptr;
            b.bytes = 0;
        }
        const size_t want = std::max<size_t>(bytes, 256);
        if (hipMalloc(&b.p, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SBR_ERR_OOM, "workspace allocation of " + std::to_string(want) + " bytes failed");
        }
        b.bytes = want;
    }
    *out = b.p;
    return SBR_OK;
}

int Workspace::get_pinned(size_t bytes, void **out)
{
    if (pinned_bytes < bytes) {
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        pinned_bytes = 0;
        if (hipHostMalloc(&pinned, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SBR_ERR_OOM, "pinned host allocation failed");
        }
        pinned_bytes = bytes;
    }
    *out = pinned;
    return SBR_OK;
}

// workspace slots
enum Slot {
    W_COUNTERS = 0,
    W_QA = 1,   // 6 buffers: 1..6
    W_QB = 7,   // 7..12
    W_REC = 13, // 13 (14..16 unused)
    W_PLANS = 17,
    W_TILEBASE = 18,
    W_BASIS = 20,
    W_KF = 21,
    W_PARTIAL = 22,
    W_SPILL = 23,
    W_MASK = 24,
    W_TUNE = 25,
    W_HELD = 26,  // record-slot bytes
    W_LIVE = 27,     // live tiles of a chunk
    W_LIVEBLK = 28,  // their per-block offsets and count
};

static int get_queue(Workspace *ws, int first, size_t cap, RayQueue &q)
{
    void *p[6];
    const size_t sz[6] = {16, 16, 16, 16, 16, 16};
    for (int i = 0; i < 6; ++i) {
        int rc = ws->get(first + i, sz[i] * cap, &p[i]);
        if (rc) return rc;
    }
    q.s0 = static_cast<float4 *>(p[0]);
    q.s1 = static_cast<float4 *>(p[1]);
    q.s2 = static_cast<float4 *>(p[2]);
    q.s3 = static_cast<float4 *>(p[3]);
    q.s4 = static_cast<double2 *>(p[4]);
    q.s5 = static_cast<double2 *>(p[5]);
    return SBR_OK;
}

static int get_records(Workspace *ws, size_t cap, Records &r)
{
    void *pr, *pv;
    int rc;
    if ((rc = ws->get(W_REC, sizeof(Rec) * cap, &pr)) ||
        (rc = ws->get(W_HELD, 4 * static_cast<size_t>(held_words(static_cast<int64_t>(cap))), &pv)))
        return rc;
    r.rec = static_cast<Rec *>(pr);
    r.held = static_cast<uint8_t *>(pv);
    return SBR_OK;
}

// Counter block (layout in sbr_internal.hpp).
struct Counters {
    CounterPtrs p;
    void *base;
    size_t bytes;
};

static int get_counters(Workspace *ws, Counters &c)
{
    const size_t bytes = kCounterBytes;
    void *p;
    int rc = ws->get(W_COUNTERS, bytes, &p);
    if (rc) return rc;
    char *b = static_cast<char *>(p);
    c.p.stat = reinterpret_cast<unsigned long long *>(b);
    c.p.q_cnt = reinterpret_cast<uint32_t *>(b + kStatBytes);
    c.p.claim = c.p.q_cnt + static_cast<size_t>(kLineU32) * kQcnt;
    c.base = p;
    c.bytes = bytes;
    return SBR_OK;
}

static int schedule_of(uint32_t flags) { return (flags & SBR_OPT_WAVEFRONT) ? kScheduleWavefront : kScheduleStream; }

// Launches every bounce of one trace: one streaming launch, or one launch
// per bounce with the two queues swapped in between.  ev (nullable) receives
// an event after each launch (ev[0] must already be recorded).
int run_trace(hipStream_t s, TraceArgs &a, RayQueue qa, RayQueue qb, std::vector<hipEvent_t> *ev)
{
    int rc;
    if (a.schedule == kScheduleStream) {
        if ((rc = launch_trace(s, a, 1))) return rc;
        if (ev) SBR_HIP(hipEventRecord((*ev)[1], s));
        return SBR_OK;
    }
    a.q_in = qb;
    a.q_out = qa;
    for (int b = 1; b <= a.bmax; ++b) {
        if (b > 1) std::swap(a.q_in, a.q_out);
        if ((rc = launch_trace(s, a, b))) return rc;
        if (ev) SBR_HIP(hipEventRecord((*ev)[b], s));
    }
    return SBR_OK;
}

size_t spill_words(const sbr_bvh *bvh, int blocks)
{
    // enough for either traversal (the binary tree, or its BVH4 copy when there is one)
    int extra = 1;
    for (int wide = 0; wide <= (bvh->nodes4 ? 1 : 0); ++wide)
        if (trace_needs_spill(bvh, wide != 0)) extra = std::max(extra, stack_need(bvh, wide != 0) + 2 - trace_stack_lds());
    return static_cast<size_t>(extra) * blocks * trace_block_threads();
}

static int get_spill(sbr_ctx *ctx, const sbr_bvh *bvh, int blocks, int32_t **spill)
{
    const size_t n = spill_words(bvh, blocks);
    void *p;
    int rc = ctx->ws->get(W_SPILL, 4 * n, &p);
    if (rc) return rc;
    *spill = static_cast<int32_t *>(p);
    return SBR_OK;
}

sbr_tune default_tune()
{
    sbr_tune t;
    t.struct_size = sizeof(sbr_tune);
    t.schedule = kScheduleStream;
    t.tile_w = 8;
    t.claim_tiles = 0;  // automatic (auto_claim_tiles)
    t.refill_min = 64;
    t.blocks_per_cu = 0;
    t.chunk_log2 = 0;  // automatic (auto_sweep_chunk_log2; batches kDefaultChunkLog2)
    t.reserved = 0;
    return t;
}

int auto_chunk_log2(size_t held_bytes)
{
    const size_t need = (size_t(1) << 30) * (sizeof(Rec) + 1);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return kDefaultChunkLog2;
    }
    return (fr + held_bytes) / 4 >= need ? 30 : kDefaultChunkLog2;
}

// The sweep's: the record buffers its workspace already holds count as free.
static int auto_sweep_chunk_log2(Workspace *ws)
{
    size_t held = 0;
    for (const int w : {W_REC, W_HELD})
        if (w < static_cast<int>(ws->bufs.size())) held += ws->bufs[w].bytes;
    return auto_chunk_log2(held);
}

int auto_claim_tiles(const sbr_bvh *bvh)
{
    const int64_t bytes = bvh->n_nodes * static_cast<int64_t>(sizeof(BNode)) +
                          bvh->n_tris * static_cast<int64_t>(sizeof(BTri));
    return bytes > kL2BytesPerXcd ? 1 : 2;
}

int normalize_tune(sbr_tune &t)
{
    int rc = check_tune(t);
    if (rc) return rc;
    if (t.chunk_log2 == 0) t.chunk_log2 = kDefaultChunkLog2;
    return SBR_OK;
}

void fill_plan(const sbr_angle_plan &ap, double ds, int tile_w, AnglePlan &p)
{
    const int th = 64 / tile_w;
    for (int i = 0; i < 3; ++i) {
        p.k[i] = ap.k_hat[i];
        p.u[i] = ap.phi_hat[i];
        p.v[i] = ap.theta_hat[i];
        p.d32[i] = static_cast<float>(ap.k_hat[i]);
        p.eH32[i] = static_cast<float>(ap.phi_hat[i]);
        p.eV32[i] = static_cast<float>(ap.theta_hat[i]);
    }
    p.uc = ap.uc;
    p.vc = ap.vc;
    p.s0 = ap.s0;
    p.ds = ds;
    p.nu = static_cast<int32_t>(ap.nu);
    p.nv = static_cast<int32_t>(ap.nv);
    p.tu = static_cast<int32_t>((ap.nu + tile_w - 1) / tile_w);
    p.tv = static_cast<int32_t>((ap.nv + th - 1) / th);
    p.tile_base = 0;
    p.rec_base = 0;
    p.root = 0;
    p.eps = 0.f;
    p.pbox = 0.f;
    p.mcu = 0;
    p.mask_base = 0;
    p.mwork_base = 0;
    p.node_cnt = 0;
    p.mslack = 0.f;
}

void mask_plan(AnglePlan &p, const double bbox[6], int64_t node_cnt)
{
    p.mcu = (p.nu + kMaskCell - 1) >> kMaskShift;
    p.node_cnt = static_cast<int32_t>(node_cnt);
    // A ray passes a (padded) box test only if its line comes within a few
    // float32 rounding errors of the box: of the order 2^-24 times the
    // magnitudes of the origin and of the box corners.  The margin takes 64
    // times that bound, plus half a ray spacing.
    double r = 0.0;
    for (int i = 0; i < 3; ++i) r += std::max(std::fabs(bbox[i]), std::fabs(bbox[3 + i]));
    const double ro = std::fabs(p.uc) + std::fabs(p.vc) + std::fabs(p.s0) + 0.5 * (double(p.nu) + p.nv) * p.ds;
    p.mslack = static_cast<float>(0.5 + 64.0 * 0x1p-24 * (r + ro) / p.ds);
}

int scene_plan(AnglePlan &p, int32_t root, float eps, const double bbox[6], double diag, int64_t node_cnt)
{
    const SceneScale sc = scene_scale(bbox, diag);
    p.root = root;
    p.eps = eps;
    p.pbox = sc.pbox;
    mask_plan(p, bbox, node_cnt);
    // origins are affine in (i, j): the grid's corners bound them
    double om = 0.0;
    for (int c = 0; c < 4; ++c) {
        const double i = (c & 1) ? p.nu - 1 : 0, j = (c & 2) ? p.nv - 1 : 0;
        const double ui = p.uc + ((i + 0.5) - 0.5 * static_cast<double>(p.nu)) * p.ds;
        const double vj = p.vc + ((j + 0.5) - 0.5 * static_cast<double>(p.nv)) * p.ds;
        for (int a = 0; a < 3; ++a) om = std::max(om, std::fabs((ui * p.u[a] + vj * p.v[a]) + p.s0 * p.k[a]));
    }
    if (!(om <= sc.obound * (1.0 - 0x1p-20)))
        return fail(SBR_ERR_SAMPLING, "ray spacing too coarse for the scene: aperture origins beyond its rounding bound");
    return SBR_OK;
}

void mask_layout(AnglePlan *plans, int64_t a0, int64_t a1, int64_t &bytes, int64_t &units)
{
    bytes = 0;
    units = 0;
    for (int64_t a = a0; a < a1; ++a) {
        AnglePlan &p = plans[a];
        const int64_t mcv = (p.nv + kMaskCell - 1) >> kMaskShift;
        p.mask_base = bytes;
        p.mwork_base = units;
        bytes += (int64_t(p.mcu) * mcv + 3) & ~int64_t(3);
        units += p.node_cnt;
    }
}

double uniform_step(const double *kf, int n)
{
    if (n < 2) return 0.0;
    const double dk = (kf[n - 1] - kf[0]) / (n - 1);
    if (!(dk != 0.0)) return 0.0;
    for (int i = 1; i < n - 1; ++i)
        if (std::fabs(kf[i] - (kf[0] + i * dk)) > 1e-14 * std::fabs(kf[i])) return 0.0;
    return dk;
}

int log2i(int x)
{
    int s = 0;
    while ((1 << s) < x) ++s;
    return s;
}

void fill_stats(sbr_stats *st, const unsigned long long *hstat, int bmax, int64_t rays, bool drop_trapped,
                int64_t chunks)
{
    st->chunks += chunks;
    st->queries += static_cast<int64_t>(hstat[0]);
    st->trapped += static_cast<int64_t>(hstat[1]);
    for (int b = 1; b <= bmax && b <= SBR_MAX_BOUNCES; ++b) st->hits[b] += static_cast<int64_t>(hstat[8 + b]);
    st->queries_bounce[1] += rays;
    for (int b = 2; b <= bmax; ++b) st->queries_bounce[b] += static_cast<int64_t>(hstat[8 + b - 1]);
    if (drop_trapped) st->queries_bounce[bmax] += static_cast<int64_t>(hstat[8 + bmax]);
    // a ray is valid when it hit at bounce 1 and was not dropped as trapped
    st->valid += static_cast<int64_t>(hstat[8 + 1]) - static_cast<int64_t>(hstat[1]);
    for (int i = 0; i < 6; ++i) st->trav[i] += static_cast<int64_t>(hstat[2 + i]);
    st->masked += static_cast<int64_t>(hstat[kStatMasked]);
}

}  // namespace sbr

using namespace sbr;

// ---------------------------------------------------------------- library
extern "C" int sbr_version(void) { return SBR_ABI_VERSION; }

extern "C" const char *sbr_last_error(void) { return g_err.c_str(); }

extern "C" int sbr_create(sbr_ctx **out, int device, void *hip_stream)
{
    if (!out) return fail(SBR_ERR_INVALID_ARG, "sbr_create: out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return fail(SBR_ERR_INVALID_ARG, "sbr_create: no HIP device with index " + std::to_string(device));
    }
    SBR_HIP(hipSetDevice(device));
    sbr_ctx *c = new (std::nothrow) sbr_ctx();
    if (!c) return fail(SBR_ERR_OOM, "sbr_create: out of host memory");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = new (std::nothrow) Workspace();
    if (hipGetDeviceProperties(&c->prop, device) != hipSuccess || !c->ws) {
        delete c->ws;
        delete c;
        return fail(SBR_ERR_HIP, "sbr_create: hipGetDeviceProperties failed");
    }
    // the no-alloc trace's static scratch: this device's address, looked up once
    int rc = noalloc_scratch_setup(device);
    if (rc) {
        delete c->ws;
        delete c;
        return rc;
    }
    *out = c;
    return SBR_OK;
}

extern "C" int sbr_set_stream(sbr_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(SBR_ERR_INVALID_ARG, "sbr_set_stream: NULL context");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SBR_OK;
}

extern "C" int sbr_synchronize(sbr_ctx *ctx)
{
    if (!ctx) return fail(SBR_ERR_INVALID_ARG, "sbr_synchronize: NULL context");
    SBR_HIP(hipSetDevice(ctx->device));
    SBR_HIP(hipStreamSynchronize(ctx->stream));
    return SBR_OK;
}

extern "C" void sbr_destroy(sbr_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx->ws;
    delete ctx;
}

// ---------------------------------------------------------------- BVH
extern "C" int sbr_build_bvh(sbr_ctx *ctx, const float *verts, int64_t n_verts, const int32_t *tris,
                             int64_t n_tris, const sbr_bvh_opts *opts, sbr_bvh **out)
{
    if (!ctx || !out || !verts || !tris) return fail(SBR_ERR_INVALID_ARG, "sbr_build_bvh: NULL argument");
    *out = nullptr;
    if (n_tris < 1 || n_tris > (int64_t(1) << 28) || n_verts < 3 || n_verts > (int64_t(1) << 31) - 1)
        return fail(SBR_ERR_INVALID_ARG, "sbr_build_bvh: n_tris must be in [1, 2^28] and n_verts >= 3");
    int mem = SBR_MEM_HOST, leaf = 4, builder = SBR_BUILD_LBVH;
    if (opts) {
        if (opts->struct_size < sizeof(sbr_bvh_opts))
            return fail(SBR_ERR_INVALID_ARG, "sbr_build_bvh: opts->struct_size too small");
        mem = opts->mem;
        if (opts->leaf_size != 0) leaf = opts->leaf_size;
        builder = opts->builder;
    }
    if (builder != SBR_BUILD_LBVH && builder != SBR_BUILD_SAH && builder != SBR_BUILD_PLOC)
        return fail(SBR_ERR_INVALID_ARG, "sbr_build_bvh: unknown builder");
    if (leaf < 1 || leaf > 4) return fail(SBR_ERR_INVALID_ARG, "sbr_build_bvh: leaf_size must be in [0, 4]");
    if (mem != SBR_MEM_HOST && mem != SBR_MEM_DEVICE)
        return fail(SBR_ERR_INVALID_ARG, "sbr_build_bvh: opts->mem must be SBR_MEM_HOST or SBR_MEM_DEVICE");
    SBR_HIP(hipSetDevice(ctx->device));
    std::vector<float> hv;
    std::vector<int32_t> ht;
    const float *V = verts;
    const int32_t *T = tris;
    if (mem == SBR_MEM_DEVICE) {
        hv.resize(3 * n_verts);
        ht.resize(3 * n_tris);
        SBR_HIP(hipMemcpyAsync(hv.data(), verts, 12 * n_verts, hipMemcpyDeviceToHost, ctx->stream));
        SBR_HIP(hipMemcpyAsync(ht.data(), tris, 12 * n_tris, hipMemcpyDeviceToHost, ctx->stream));
        SBR_HIP(hipStreamSynchronize(ctx->stream));
        V = hv.data();
        T = ht.data();
    }
    PreparedMesh pm;
    int rc = prepare_mesh(V, n_verts, T, n_tris, pm);
    if (rc) return rc;
    sbr_bvh *b = new (std::nothrow) sbr_bvh();
    if (!b) return fail(SBR_ERR_OOM, "sbr_build_bvh: out of host memory");
    b->device = ctx->device;
    b->n_tris = n_tris;
    b->eps = pm.eps;
    b->diag = pm.diag;
    std::memcpy(b->bbox, pm.bbox, sizeof(pm.bbox));
    b->leaf_size = leaf;
    rc = builder == SBR_BUILD_SAH    ? build_sah(ctx, pm, leaf, b)
         : builder == SBR_BUILD_PLOC ? build_ploc(ctx, pm, leaf, b)
                                     : build_lbvh(ctx, pm, leaf, b);
    if (rc) {
        sbr_free_bvh(b);
        return rc;
    }
    b->host_normals = pm.n;
    *out = b;
    return SBR_OK;
}

extern "C" int sbr_bvh_get_info(const sbr_bvh *bvh, sbr_bvh_info *out)
{
    if (!bvh || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_bvh_get_info: NULL argument");
    out->n_tris = bvh->n_tris;
    out->n_live = bvh->n_live;
    out->n_nodes = bvh->n_nodes;
    out->depth = bvh->depth;
    out->eps = bvh->eps;
    std::memcpy(out->bbox, bvh->bbox, sizeof(bvh->bbox));
    out->device_bytes = bvh->device_bytes;
    out->n_scenes = bvh->scenes.empty() ? 1 : static_cast<int32_t>(bvh->scenes.size());
    out->reserved = 0;
    return SBR_OK;
}

extern "C" int sbr_bvh_validate(const sbr_bvh *bvh)
{
    if (!bvh) return fail(SBR_ERR_INVALID_ARG, "sbr_bvh_validate: NULL argument");
    if (!bvh->scenes.empty()) return fail(SBR_ERR_UNSUPPORTED, "sbr_bvh_validate: a scene set is checked per scene");
    if (bvh->n_live == 0) return bvh->n_nodes == 0 ? SBR_OK : fail(SBR_ERR_INVALID_MESH, "BVH layout: nodes without triangles");
    SBR_HIP(hipSetDevice(bvh->device));
    std::vector<BNode> hn(static_cast<size_t>(bvh->n_nodes));
    std::vector<BTri> ht(static_cast<size_t>(bvh->n_live));
    SBR_HIP(hipMemcpy(hn.data(), bvh->nodes, sizeof(BNode) * hn.size(), hipMemcpyDeviceToHost));
    SBR_HIP(hipMemcpy(ht.data(), bvh->tris, sizeof(BTri) * ht.size(), hipMemcpyDeviceToHost));
    const SceneScale sc = scene_scale(bvh->bbox, bvh->diag);
    int rc = validate_layout(hn, static_cast<int>(bvh->n_live), bvh->leaf_size, bvh->depth, &ht, bvh->n_tris, &sc);
    if (rc || !bvh->nodes4) return rc;
    std::vector<BNode4> hw(static_cast<size_t>(bvh->n_nodes4));
    SBR_HIP(hipMemcpy(hw.data(), bvh->nodes4, sizeof(BNode4) * hw.size(), hipMemcpyDeviceToHost));
    return validate_wide(hn, hw, bvh->depth4);
}

extern "C" int sbr_bvh_quality_of(const sbr_bvh *bvh, sbr_bvh_quality *out)
{
    if (!bvh || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_bvh_quality_of: NULL argument");
    if (!bvh->scenes.empty()) return fail(SBR_ERR_UNSUPPORTED, "sbr_bvh_quality_of: a scene set is measured per scene");
    *out = sbr_bvh_quality{};
    if (bvh->n_nodes == 0) return SBR_OK;
    SBR_HIP(hipSetDevice(bvh->device));
    std::vector<BNode> hn(static_cast<size_t>(bvh->n_nodes));
    SBR_HIP(hipMemcpy(hn.data(), bvh->nodes, sizeof(BNode) * hn.size(), hipMemcpyDeviceToHost));
    layout_quality(hn, *out);
    return SBR_OK;
}

extern "C" int sbr_bvh_normals(const sbr_bvh *bvh, float *out_host)
{
    if (!bvh || !out_host) return fail(SBR_ERR_INVALID_ARG, "sbr_bvh_normals: NULL argument");
    std::memcpy(out_host, bvh->host_normals.data(), sizeof(float) * bvh->host_normals.size());
    return SBR_OK;
}

extern "C" void sbr_free_bvh(sbr_bvh *bvh)
{
    if (!bvh) return;
    (void)hipSetDevice(bvh->device);
    if (!bvh->blocks.empty()) {
        (void)hipDeviceSynchronize();  // no kernel may still read the arrays when their blocks are handed on
        for (const auto &b : bvh->blocks) device_block_put(bvh->device, b.first, b.second);
    }
    delete bvh;
}

// ---------------------------------------------------------------- trace
// sbr_trace and sbr_trace_noalloc.  noalloc: the counter block lives in the
// library's static per-device scratch, cleared by a fill kernel; nothing is
// allocated (no workspace growth, no events), and what would need more
// memory than the scratch holds (the wavefront schedule's queues, a stack
// spill for deep trees) is refused.
static int trace_impl(const char *fn, sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_rays *rays, int64_t n_rays,
                      int max_bounces, const sbr_trace_opts *opts, sbr_hits *out, sbr_stats *stats, bool noalloc)
{
    const auto t_start = std::chrono::steady_clock::now();
    const std::string f(fn);
    if (!ctx || !bvh || !rays || !out) return fail(SBR_ERR_INVALID_ARG, f + ": NULL argument");
    if (!rays->o || !rays->d || !rays->eH || !rays->eV)
        return fail(SBR_ERR_INVALID_ARG, f + ": rays->o, d, eH and eV are required");
    if (n_rays < 1 || n_rays > 2147483647LL) return fail(SBR_ERR_INVALID_ARG, f + ": n_rays out of range");
    if (max_bounces < 1 || max_bounces > SBR_MAX_BOUNCES)
        return fail(SBR_ERR_INVALID_ARG, f + ": max_bounces must be in [1, " + std::to_string(SBR_MAX_BOUNCES) + "]");
    uint32_t flags = 0;
    double k[3] = {0, 0, -1};
    if (opts) {
        if (opts->struct_size < sizeof(sbr_trace_opts))
            return fail(SBR_ERR_INVALID_ARG, f + ": opts->struct_size too small");
        flags = opts->flags;
        for (int a = 0; a < 3; ++a) k[a] = opts->k_hat[a];
    }
    if (bvh->device != ctx->device) return fail(SBR_ERR_INVALID_ARG, f + ": BVH lives on another device");
    if (!bvh->scenes.empty()) return fail(SBR_ERR_INVALID_ARG, f + ": a multi-scene set serves batches only");
    SBR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    Workspace *ws = ctx->ws;
    int rc;
    Counters cn;
    RayQueue qa{}, qb{};
    int32_t *spill;
    const int sched = schedule_of(flags);
    if ((flags & SBR_OPT_FP64_TRAVERSE) && sched != kScheduleStream)
        return fail(SBR_ERR_UNSUPPORTED, f + ": SBR_OPT_FP64_TRAVERSE runs on the streaming schedule only");
    sbr_tune tune = default_tune();
    tune.claim_tiles = auto_claim_tiles(bvh);
    const int blocks = trace_persistent_blocks(ctx, tune.blocks_per_cu);
    if (noalloc) {
        if (sched != kScheduleStream)
            return fail(SBR_ERR_UNSUPPORTED, f + ": the wavefront schedule needs ray queues beyond the static scratch");
        if (flags & SBR_OPT_BVH4)
            return fail(SBR_ERR_UNSUPPORTED, f + ": SBR_OPT_BVH4 may need to build the tree's wide copy");
        if (trace_needs_spill(bvh, false))
            return fail(SBR_ERR_UNSUPPORTED,
                        f + ": the tree (depth " + std::to_string(bvh->depth) + ") needs more traversal stack "
                            "than the on-chip one; the static scratch holds no stack spill (use sbr_trace)");
        if ((rc = noalloc_counters(ctx->device, cn.p, &cn.base, &cn.bytes))) return rc;
        spill = nullptr;  // never read: the tree fits the on-chip stack
    } else {
        if ((rc = ensure_wide(ctx, bvh, flags, sched))) return rc;
        if ((rc = get_counters(ws, cn)) || (rc = get_spill(ctx, bvh, blocks, &spill))) return rc;
        if (sched == kScheduleWavefront &&
            ((rc = get_queue(ws, W_QA, n_rays, qa)) || (rc = get_queue(ws, W_QB, n_rays, qb))))
            return rc;
    }
    if (bvh->n_live == 0) return fail(SBR_ERR_INVALID_ARG, f + ": the mesh has no non-degenerate triangle");
    if (noalloc) {
        if ((rc = launch_zero_u32(s, static_cast<uint32_t *>(cn.base), static_cast<int64_t>(cn.bytes / 4)))) return rc;
    } else {
        SBR_HIP(hipMemsetAsync(cn.base, 0, cn.bytes, s));
    }
    const bool want_stats = stats != nullptr;
    const bool timed = want_stats && !noalloc;
    std::vector<hipEvent_t> ev;
    if (timed) {
        ev.resize(max_bounces + 1);
        for (auto &e : ev) SBR_HIP(hipEventCreate(&e));
        SBR_HIP(hipEventRecord(ev[0], s));
    }
    TraceArgs a{};
    a.bvh = bvh;
    a.bmax = max_bounces;
    a.flags = flags;
    a.schedule = sched;
    a.tile_shift = log2i(tune.tile_w);
    a.claim_tiles = tune.claim_tiles;
    a.refill_min = tune.refill_min;
    a.blocks = blocks;
    a.rays = rays;
    a.n_rays = n_rays;
    a.hits = out;
    for (int i = 0; i < 3; ++i) a.k_hat[i] = k[i];
    a.ctrs = cn.p;
    a.spill = spill;
    if ((rc = run_trace(s, a, qa, qb, timed ? &ev : nullptr))) return rc;
    if (want_stats || (flags & SBR_OPT_SYNC)) {
        unsigned long long hstat[kStatU64];
        SBR_HIP(hipMemcpyAsync(hstat, cn.p.stat, sizeof(hstat), hipMemcpyDeviceToHost, s));
        SBR_HIP(hipStreamSynchronize(s));
        if (want_stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->rays = n_rays;
            fill_stats(stats, hstat, max_bounces, n_rays, (flags & SBR_OPT_DROP_TRAPPED) != 0,
                       sched == kScheduleStream ? 1 : 0);
            const int nl = !timed ? 0 : sched == kScheduleStream ? 1 : max_bounces;
            for (int b = 1; b <= nl; ++b) {
                float ms = 0;
                SBR_HIP(hipEventElapsedTime(&ms, ev[b - 1], ev[b]));
                if (sched == kScheduleWavefront) stats->ms_bounce[b] = ms;
                stats->ms_trace += ms;
            }
            stats->ms_total =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            for (auto &e : ev) (void)hipEventDestroy(e);
        }
    }
    return SBR_OK;
}

extern "C" int sbr_trace(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_rays *rays, int64_t n_rays, int max_bounces,
                         const sbr_trace_opts *opts, sbr_hits *out, sbr_stats *stats)
{
    return trace_impl("sbr_trace", ctx, bvh, rays, n_rays, max_bounces, opts, out, stats, false);
}

extern "C" int sbr_trace_noalloc(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_rays *rays, int64_t n_rays,
                                 int max_bounces, const sbr_trace_opts *opts, sbr_hits *out, sbr_stats *stats)
{
    return trace_impl("sbr_trace_noalloc", ctx, bvh, rays, n_rays, max_bounces, opts, out, stats, true);
}

// ---------------------------------------------------------------- PO
static int basis_from_desc(const sbr_po_desc *d, double *out)
{
    for (int a = 0; a < 3; ++a) {
        out[a] = d->k_hat[a];
        out[3 + a] = d->theta_hat[a];
        out[6 + a] = d->phi_hat[a];
    }
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(out[i])) return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: non-finite basis");
    return SBR_OK;
}

extern "C" int sbr_po_integrate(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_hits *hits, int64_t n_rays,
                                const sbr_po_desc *desc, const double *freqs_hz, int n_freq, double *A_out)
{
    if (!ctx || !bvh || !hits || !desc || !freqs_hz || !A_out)
        return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: NULL argument");
    if (desc->struct_size < sizeof(sbr_po_desc))
        return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: desc->struct_size too small");
    if (!hits->n_bounce || !hits->tri_first || !hits->tri_last || !hits->flags || !hits->D || !hits->d_last ||
        !hits->eH_last || !hits->eV_last)
        return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: hits lacks a required array");
    if (n_rays < 1 || n_rays > 2147483647LL) return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: n_rays out of range");
    if (n_freq < 1 || n_freq > 4096) return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: n_freq must be in [1, 4096]");
    if (desc->mode != SBR_MODE_VECTOR && desc->mode != SBR_MODE_PAPER)
        return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: unknown mode");
    if (!(desc->dA > 0.0)) return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: dA must be positive");
    for (int f = 0; f < n_freq; ++f)
        if (!(freqs_hz[f] > 0.0) || !std::isfinite(freqs_hz[f]))
            return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: frequencies must be positive");
    if (!bvh->scenes.empty())
        return fail(SBR_ERR_INVALID_ARG, "sbr_po_integrate: a multi-scene set serves batches only");
    SBR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    Workspace *ws = ctx->ws;
    int rc;
    PoAngle ang{};
    if ((rc = basis_from_desc(desc, ang.basis))) return rc;
    ang.dA = desc->dA;
    ang.rec_base = 0;
    ang.rec_cnt = n_rays;
    ang.unit_base = 0;
    ang.part_base = 0;
    ang.out_base = 0;
    ang.kf_off = 0;
    ang.n_f = n_freq;
    {
        std::vector<double> kfv(n_freq);
        for (int f = 0; f < n_freq; ++f) kfv[f] = 2.0 * kPi * freqs_hz[f] / kC0;
        ang.dk = uniform_step(kfv.data(), n_freq);
    }
    const int64_t units = po_units(n_rays);
    Records rec;
    void *pang, *pkf, *ppart, *ph;
    const size_t host_bytes = sizeof(PoAngle) + 8 * static_cast<size_t>(n_freq);
    if ((rc = get_records(ws, n_rays, rec)) || (rc = ws->get(W_BASIS, sizeof(PoAngle), &pang)) ||
        (rc = ws->get(W_KF, 8 * n_freq, &pkf)) ||
        (rc = ws->get(W_PARTIAL, 64 * static_cast<size_t>(units) * n_freq, &ppart)) ||
        (rc = ws->get_pinned(host_bytes, &ph)))
        return rc;
    SBR_HIP(hipStreamSynchronize(s));  // the pinned staging buffer may still feed an earlier copy
    std::memcpy(ph, &ang, sizeof(PoAngle));
    double *hkf = reinterpret_cast<double *>(static_cast<char *>(ph) + sizeof(PoAngle));
    for (int f = 0; f < n_freq; ++f) hkf[f] = 2.0 * kPi * freqs_hz[f] / kC0;
    SBR_HIP(hipMemcpyAsync(pang, ph, sizeof(PoAngle), hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(pkf, hkf, 8 * n_freq, hipMemcpyHostToDevice, s));
    if ((rc = launch_pack_hits(s, hits, n_rays, rec))) return rc;
    PoArgs pa{};
    pa.bvh = bvh;
    pa.rec = rec;
    pa.ang = static_cast<const PoAngle *>(pang);
    pa.n_angles = 1;
    pa.n_units = units;
    pa.max_nf = n_freq;
    pa.kinds = po_kind(ang.dk);
    pa.mode = desc->mode;
    pa.kf = static_cast<const double *>(pkf);
    pa.partial = static_cast<long long *>(ppart);
    if ((rc = launch_po(s, pa)) || (rc = launch_po_finalize(s, pa, A_out, nullptr))) return rc;
    return SBR_OK;
}

// ---------------------------------------------------------------- sweep
extern "C" int sbr_default_tune(sbr_tune *out)
{
    if (!out) return fail(SBR_ERR_INVALID_ARG, "sbr_default_tune: NULL argument");
    *out = default_tune();
    return SBR_OK;
}

extern "C" int sbr_plan_angle(const double bbox[6], double theta_deg, double phi_deg, double ds, double eta,
                              sbr_angle_plan *out)
{
    if (!bbox || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_plan_angle: NULL argument");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(bbox[i])) return fail(SBR_ERR_INVALID_ARG, "sbr_plan_angle: non-finite bbox");
    return plan_angle(bbox, theta_deg, phi_deg, ds, eta, *out);
}


extern "C" int sbr_rcs_sweep(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_sweep *sw, double *A_out,
                             double *sigma_dbsm, sbr_stats *stats)
{
    const auto t_start = std::chrono::steady_clock::now();
    if (!ctx || !bvh || !sw || !A_out) return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: NULL argument");
    if (sw->struct_size < sizeof(sbr_sweep))
        return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: sweep->struct_size too small");
    if (!sw->theta_deg || !sw->phi_deg || !sw->freqs_hz)
        return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: NULL angle or frequency array");
    if (sw->n_angles < 1 || sw->n_angles > (int64_t(1) << 24))
        return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: n_angles must be in [1, 2^24]");
    if (sw->n_freq < 1 || sw->n_freq > 4096)
        return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: n_freq must be in [1, 4096]");
    if (sw->max_bounces < 1 || sw->max_bounces > SBR_MAX_BOUNCES)
        return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: max_bounces must be in [1, " + std::to_string(SBR_MAX_BOUNCES) + "]");
    if (sw->mode != SBR_MODE_VECTOR && sw->mode != SBR_MODE_PAPER)
        return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: unknown mode");
    if (bvh->device != ctx->device) return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: BVH lives on another device");
    double fmax = 0.0;
    for (int f = 0; f < sw->n_freq; ++f) {
        if (!(sw->freqs_hz[f] > 0.0) || !std::isfinite(sw->freqs_hz[f]))
            return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: frequencies must be positive and finite");
        fmax = std::max(fmax, sw->freqs_hz[f]);
    }
    double ds = sw->ds;
    if (!(ds > 0.0)) {
        if (!(sw->samples_per_lambda > 0.0))
            return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: give ds or samples_per_lambda");
        ds = kC0 / fmax / sw->samples_per_lambda;
    }
    // sampling rule of Sec. 4: ds <= lambda / 5 at the highest frequency
    if (ds > (kC0 / fmax / 5.0) * (1.0 + 1e-12) && !(sw->flags & SBR_OPT_ALLOW_UNDERSAMPLING))
        return fail(SBR_ERR_SAMPLING, "sbr_rcs_sweep: ray spacing " + std::to_string(ds) +
                                          " m exceeds lambda/5 at the highest frequency");
    const double eta = sw->eta < 0.0 ? 0.1 : sw->eta;
    sbr_tune tune = default_tune();
    if (sw->tune) {
        if (sw->tune->struct_size < sizeof(sbr_tune))
            return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: tune->struct_size too small");
        tune = *sw->tune;
    }
    if (sw->flags & SBR_OPT_WAVEFRONT) tune.schedule = kScheduleWavefront;
    if (tune.chunk_log2 == 0) {
        SBR_HIP(hipSetDevice(ctx->device));
        tune.chunk_log2 = auto_sweep_chunk_log2(ctx->ws);
    }
    int rc0 = normalize_tune(tune);
    if (rc0) return rc0;
    if (tune.claim_tiles == 0) tune.claim_tiles = auto_claim_tiles(bvh);
    const int tw = tune.tile_w;
    const int64_t chunk_cap = int64_t(1) << tune.chunk_log2;
    if (bvh->n_live == 0) return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: the mesh has no non-degenerate triangle");
    if (!bvh->scenes.empty()) return fail(SBR_ERR_INVALID_ARG, "sbr_rcs_sweep: a multi-scene set serves batches only");
    SBR_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    Workspace *ws = ctx->ws;
    const int64_t na = sw->n_angles;
    const int nf = sw->n_freq;
    int rc;

    // plans of every angle (host, float64)
    std::vector<AnglePlan> plans(na);
    std::vector<PoAngle> pang(na);
    for (int64_t a = 0; a < na; ++a) {
        sbr_angle_plan ap;
        if ((rc = plan_angle(bvh->bbox, sw->theta_deg[a], sw->phi_deg[a], ds, eta, ap))) return rc;
        if (ap.nu * ap.nv > (int64_t(1) << 31) - 1) return fail(SBR_ERR_OVERFLOW, "sbr_rcs_sweep: too many rays per angle");
        AnglePlan &p = plans[a];
        fill_plan(ap, ds, tw, p);
        if ((rc = scene_plan(p, 0, bvh->eps, bvh->bbox, bvh->diag, bvh->n_nodes))) return rc;
        PoAngle &q = pang[a];
        for (int i = 0; i < 3; ++i) {
            q.basis[i] = ap.k_hat[i];
            q.basis[3 + i] = ap.theta_hat[i];
            q.basis[6 + i] = ap.phi_hat[i];
        }
        q.dA = ds * ds;
        q.rec_cnt = ap.nu * ap.nv;
        q.out_base = a * nf;
        q.kf_off = 0;
        q.n_f = nf;
        q.dk = 0.0;
    }
    {
        std::vector<double> kfv(nf);
        for (int f = 0; f < nf; ++f) kfv[f] = 2.0 * kPi * sw->freqs_hz[f] / kC0;
        const double dk = uniform_step(kfv.data(), nf);
        for (auto &q : pang) q.dk = dk;
    }
    // chunks of consecutive angles holding at most chunk_cap rays (or one angle)
    std::vector<int64_t> cstart;
    std::vector<int64_t> chunk_units, chunk_mask_bytes, chunk_mask_units;
    int64_t max_chunk_rays = 0, max_chunk_units = 0, max_mask_bytes = 0, max_chunk_tiles = 0;
    {
        int64_t a = 0;
        while (a < na) {
            cstart.push_back(a);
            int64_t rays = 0, tiles = 0, units = 0, b = a;
            while (b < na) {
                const int64_t r = int64_t(plans[b].nu) * plans[b].nv;
                if (b > a && rays + r > chunk_cap) break;
                plans[b].tile_base = tiles;
                plans[b].rec_base = rays;
                pang[b].rec_base = rays;
                pang[b].unit_base = units;
                pang[b].part_base = units * nf;
                tiles += int64_t(plans[b].tu) * plans[b].tv;
                rays += r;
                units += po_units(r);
                ++b;
            }
            chunk_units.push_back(units);
            int64_t mb = 0, mu = 0;
            mask_layout(plans.data(), a, b, mb, mu);
            chunk_mask_bytes.push_back(mb);
            chunk_mask_units.push_back(mu);
            max_mask_bytes = std::max(max_mask_bytes, mb);
            max_chunk_rays = std::max(max_chunk_rays, rays);
            max_chunk_units = std::max(max_chunk_units, units);
            max_chunk_tiles = std::max(max_chunk_tiles, tiles);
            a = b;
        }
        cstart.push_back(na);
    }
    const int n_chunks = static_cast<int>(cstart.size()) - 1;

    // device buffers
    Counters cn;
    RayQueue qa{}, qb{};
    Records rec;
    int32_t *spill;
    void *dplans, *dtile, *dang, *dkf, *dpart, *hpin, *dmask = nullptr;
    const int sched = tune.schedule;
    if ((sw->flags & SBR_OPT_FP64_TRAVERSE) && sched != kScheduleStream)
        return fail(SBR_ERR_UNSUPPORTED, "sbr_rcs_sweep: SBR_OPT_FP64_TRAVERSE runs on the streaming schedule only");
    const bool use_mask = !(sw->flags & SBR_OPT_NO_MASK);
    if ((rc = ensure_wide(ctx, bvh, sw->flags, sched))) return rc;
    const int blocks = trace_persistent_blocks(ctx, tune.blocks_per_cu);
    const size_t tile_words = static_cast<size_t>(na + n_chunks);
    if ((rc = get_counters(ws, cn)) || (rc = get_records(ws, max_chunk_rays, rec)) ||
        (rc = get_spill(ctx, bvh, blocks, &spill)) || (rc = ws->get(W_PLANS, sizeof(AnglePlan) * na, &dplans)) ||
        (rc = ws->get(W_TILEBASE, 8 * tile_words, &dtile)) || (rc = ws->get(W_BASIS, sizeof(PoAngle) * na, &dang)) ||
        (rc = ws->get(W_KF, 8 * nf, &dkf)) ||
        (rc = ws->get(W_PARTIAL, 64 * static_cast<size_t>(max_chunk_units) * nf, &dpart)) ||
        (use_mask && (rc = ws->get(W_MASK, static_cast<size_t>(std::max<int64_t>((max_mask_bytes + 3) & ~int64_t(3), 4)), &dmask))))
        return rc;
    // the streaming schedule claims the live tiles of the mask
    void *dlive = nullptr, *dliveblk = nullptr;
    const bool use_live = use_mask && sched == kScheduleStream;
    if (use_live && ((rc = ws->get(W_LIVE, 4 * static_cast<size_t>(max_chunk_tiles), &dlive)) ||
                     (rc = ws->get(W_LIVEBLK, 4 * static_cast<size_t>(live_blocks(max_chunk_tiles) + 1), &dliveblk))))
        return rc;
    if (sched == kScheduleWavefront &&
        ((rc = get_queue(ws, W_QA, max_chunk_rays, qa)) || (rc = get_queue(ws, W_QB, max_chunk_rays, qb))))
        return rc;
    // host staging (pinned): plans | tile bases | PO angles | kf
    const size_t off_plans = 0;
    const size_t off_tile = off_plans + sizeof(AnglePlan) * na;
    const size_t off_ang = off_tile + 8 * tile_words;
    const size_t off_kf = off_ang + sizeof(PoAngle) * na;
    const size_t host_bytes = off_kf + 8 * nf;
    if ((rc = ws->get_pinned(host_bytes, &hpin))) return rc;
    SBR_HIP(hipStreamSynchronize(s));  // the staging buffer may still feed an earlier copy
    char *hp = static_cast<char *>(hpin);
    std::memcpy(hp + off_plans, plans.data(), sizeof(AnglePlan) * na);
    {
        int64_t *tb = reinterpret_cast<int64_t *>(hp + off_tile);
        size_t w = 0;
        for (int c = 0; c < n_chunks; ++c) {
            int64_t tiles = 0;
            for (int64_t a = cstart[c]; a < cstart[c + 1]; ++a) {
                tb[w++] = plans[a].tile_base;
                tiles = plans[a].tile_base + int64_t(plans[a].tu) * plans[a].tv;
            }
            tb[w++] = tiles;
        }
    }
    std::memcpy(hp + off_ang, pang.data(), sizeof(PoAngle) * na);
    double *hkf = reinterpret_cast<double *>(hp + off_kf);
    for (int f = 0; f < nf; ++f) hkf[f] = 2.0 * kPi * sw->freqs_hz[f] / kC0;
    SBR_HIP(hipMemcpyAsync(dplans, hp + off_plans, sizeof(AnglePlan) * na, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dtile, hp + off_tile, 8 * tile_words, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dang, hp + off_ang, sizeof(PoAngle) * na, hipMemcpyHostToDevice, s));
    SBR_HIP(hipMemcpyAsync(dkf, hp + off_kf, 8 * nf, hipMemcpyHostToDevice, s));

    const bool want_stats = stats != nullptr;
    const int bm = sw->max_bounces;
    const int epc = bm + 2;  // events per chunk: start, after each bounce, after the PO stage
    std::vector<hipEvent_t> ev;
    std::vector<int64_t> chunk_rays(n_chunks, 0);
    if (want_stats) {
        std::memset(stats, 0, sizeof(*stats));
        ev.resize(static_cast<size_t>(epc) * n_chunks);
        for (auto &e : ev) SBR_HIP(hipEventCreate(&e));
    }
    std::vector<unsigned long long> hstat(static_cast<size_t>(kStatU64) * n_chunks);
    size_t tile_off = 0;
    for (int c = 0; c < n_chunks; ++c) {
        const int64_t a0 = cstart[c], a1 = cstart[c + 1];
        const int m = static_cast<int>(a1 - a0);
        const AnglePlan *cp = static_cast<const AnglePlan *>(dplans) + a0;
        const int64_t *ctile = static_cast<const int64_t *>(dtile) + tile_off;
        tile_off += m + 1;
        int64_t n_tiles = 0, n_rays = 0;
        for (int64_t a = a0; a < a1; ++a) {
            n_tiles += int64_t(plans[a].tu) * plans[a].tv;
            n_rays += int64_t(plans[a].nu) * plans[a].nv;
        }
        chunk_rays[c] = n_rays;
        SBR_HIP(hipMemsetAsync(cn.base, 0, cn.bytes, s));
        if (want_stats) SBR_HIP(hipEventRecord(ev[epc * c], s));
        // the chunk's record slots start empty
        if ((rc = launch_zero_u32(s, reinterpret_cast<uint32_t *>(rec.held), held_words(n_rays)))) return rc;
        TraceArgs ta{};
        ta.bvh = bvh;
        ta.bmax = bm;
        ta.flags = sw->flags;
        ta.schedule = sched;
        ta.tile_shift = log2i(tw);
        ta.claim_tiles = tune.claim_tiles;
        ta.refill_min = tune.refill_min;
        ta.blocks = blocks;
        ta.plans = cp;
        ta.tile_base = ctile;
        ta.n_angles = m;
        ta.n_tiles = n_tiles;
        ta.rec = rec;
        ta.ctrs = cn.p;
        ta.spill = spill;
        if (use_mask) {
            ta.mask = static_cast<const uint8_t *>(dmask);
            if ((rc = launch_mask(s, bvh->nodes, cp, m, chunk_mask_units[c], static_cast<uint8_t *>(dmask),
                                  chunk_mask_bytes[c])))
                return rc;
            if (use_live) {
                uint32_t *blk = static_cast<uint32_t *>(dliveblk);
                if ((rc = launch_live(s, ta, static_cast<int32_t *>(dlive), blk))) return rc;
                ta.live = static_cast<const int32_t *>(dlive);
                ta.live_count = blk + live_blocks(n_tiles);
            }
        }
        std::vector<hipEvent_t> cev;
        if (want_stats) cev.assign(ev.begin() + epc * c, ev.begin() + epc * (c + 1));
        if ((rc = run_trace(s, ta, qa, qb, want_stats ? &cev : nullptr))) return rc;
        const int trace_launches = sched == kScheduleStream ? 1 : bm;
        PoArgs pa{};
        pa.bvh = bvh;
        pa.rec = rec;
        pa.rec_slots = 1;
        pa.ang = static_cast<const PoAngle *>(dang) + a0;
        pa.n_angles = m;
        pa.n_units = chunk_units[c];
        pa.max_nf = nf;
        pa.kinds = po_kind(pang[0].dk);  // one frequency list for every angle
        pa.mode = sw->mode;
        pa.kf = static_cast<const double *>(dkf);
        pa.partial = static_cast<long long *>(dpart);
        pa.fp32 = (sw->flags & SBR_OPT_FP32_PATH) ? 1 : 0;
        if ((rc = launch_po(s, pa))) return rc;
        if ((rc = launch_po_finalize(s, pa, A_out, sigma_dbsm))) return rc;
        if (want_stats) {
            SBR_HIP(hipEventRecord(ev[epc * c + trace_launches + 1], s));
            SBR_HIP(hipMemcpyAsync(hstat.data() + static_cast<size_t>(kStatU64) * c, cn.p.stat, 8 * kStatU64,
                                   hipMemcpyDeviceToHost, s));
            stats->rays += n_rays;
        }
    }
    if (want_stats || (sw->flags & SBR_OPT_SYNC)) SBR_HIP(hipStreamSynchronize(s));
    if (want_stats) {
        for (int c = 0; c < n_chunks; ++c) {
            fill_stats(stats, hstat.data() + static_cast<size_t>(kStatU64) * c, bm, chunk_rays[c],
                       (sw->flags & SBR_OPT_DROP_TRAPPED) != 0, sched == kScheduleStream ? 1 : 0);
            const int nl = sched == kScheduleStream ? 1 : bm;
            for (int b = 1; b <= nl; ++b) {
                float t = 0;
                SBR_HIP(hipEventElapsedTime(&t, ev[epc * c + b - 1], ev[epc * c + b]));
                if (sched == kScheduleWavefront) stats->ms_bounce[b] += t;
                stats->ms_trace += t;
            }
            float t2 = 0;
            SBR_HIP(hipEventElapsedTime(&t2, ev[epc * c + nl], ev[epc * c + nl + 1]));
            stats->ms_po += t2;
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
        stats->angles = na;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return SBR_OK;
}

// ---------------------------------------------------------------- autotuner
namespace {

int bucket(double x) { return x < 1.0 ? 0 : static_cast<int>(std::floor(std::log2(x))); }

std::string tune_key(const sbr_ctx *ctx, const sbr_bvh *bvh, int64_t rays_per_angle, int bmax)
{
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|t%d|r%d|b%d", ctx->prop.gcnArchName, bucket(static_cast<double>(bvh->n_live)),
                  bucket(static_cast<double>(rays_per_angle)), bmax);
    return buf;
}

// One line per entry: {"key": "...", "schedule": s, "tile_w": w, "claim_tiles": c, "refill_min": r,
// "blocks_per_cu": b, "chunk_log2": k}
bool file_lookup(const char *path, const std::string &key, sbr_tune *out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[256];
        sbr_tune t = default_tune();
        const int n = std::sscanf(line,
                                  "{\"key\": \"%255[^\"]\", \"schedule\": %d, \"tile_w\": %d, \"claim_tiles\": %d, "
                                  "\"refill_min\": %d, \"blocks_per_cu\": %d, \"chunk_log2\": %d}",
                                  k, &t.schedule, &t.tile_w, &t.claim_tiles, &t.refill_min, &t.blocks_per_cu,
                                  &t.chunk_log2);
        if (n >= 6 && key == k && normalize_tune(t) == SBR_OK) {
            *out = t;  // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    set_error("");
    return found;
}

void file_store(const char *path, const std::string &key, const sbr_tune &t)
{
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"schedule\": %d, \"tile_w\": %d, \"claim_tiles\": %d, \"refill_min\": %d, "
                 "\"blocks_per_cu\": %d, \"chunk_log2\": %d}\n",
                 key.c_str(), t.schedule, t.tile_w, t.claim_tiles, t.refill_min, t.blocks_per_cu, t.chunk_log2);
    std::fclose(f);
}

}  // namespace

namespace sbr {

bool tune_lookup(sbr_ctx *ctx, const std::string &key, sbr_tune *out)
{
    auto it = ctx->tune_cache.find(key);
    if (it != ctx->tune_cache.end()) {
        *out = it->second;
        return true;
    }
    const char *path = std::getenv("SBR_TUNE_CACHE");
    if (path && *path && file_lookup(path, key, out)) {
        ctx->tune_cache[key] = *out;
        return true;
    }
    return false;
}

void tune_store(sbr_ctx *ctx, const std::string &key, const sbr_tune &t)
{
    ctx->tune_cache[key] = t;
    const char *path = std::getenv("SBR_TUNE_CACHE");
    if (path && *path) file_store(path, key, t);
}

int size_bucket(double x) { return bucket(x); }

}  // namespace sbr

extern "C" int sbr_autotune(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_sweep *sw, sbr_tune *out)
{
    if (!ctx || !bvh || !sw || !out) return fail(SBR_ERR_INVALID_ARG, "sbr_autotune: NULL argument");
    if (!bvh->scenes.empty()) return fail(SBR_ERR_INVALID_ARG, "sbr_autotune: a multi-scene set serves batches only");
    if (sw->struct_size < sizeof(sbr_sweep)) return fail(SBR_ERR_INVALID_ARG, "sbr_autotune: sweep->struct_size too small");
    if (sw->n_angles < 1 || !sw->theta_deg || !sw->phi_deg || !sw->freqs_hz || sw->n_freq < 1)
        return fail(SBR_ERR_INVALID_ARG, "sbr_autotune: empty sweep");
    // sample of at most 16 evenly spaced angles, one frequency (the trace does not depend on it)
    const int64_t na = sw->n_angles;
    const int ns = static_cast<int>(std::min<int64_t>(na, 16));
    std::vector<double> th(ns), ph(ns);
    for (int i = 0; i < ns; ++i) {
        const int64_t a = (ns == 1) ? 0 : (i * (na - 1)) / (ns - 1);
        th[i] = sw->theta_deg[a];
        ph[i] = sw->phi_deg[a];
    }
    double fmax = 0.0;
    for (int f = 0; f < sw->n_freq; ++f) fmax = std::max(fmax, sw->freqs_hz[f]);
    sbr_sweep sub = *sw;
    sub.theta_deg = th.data();
    sub.phi_deg = ph.data();
    sub.n_angles = ns;
    sub.freqs_hz = &fmax;
    sub.n_freq = 1;
    sub.flags &= ~static_cast<uint32_t>(SBR_OPT_WAVEFRONT | SBR_OPT_SYNC);
    // rays per angle of the sample, for the cache key
    double ds = sw->ds;
    if (!(ds > 0.0)) ds = (sw->samples_per_lambda > 0.0 && fmax > 0.0) ? kC0 / fmax / sw->samples_per_lambda : 0.0;
    sbr_angle_plan ap;
    int rc = plan_angle(bvh->bbox, th[0], ph[0], ds, sw->eta < 0.0 ? 0.1 : sw->eta, ap);
    if (rc) return rc;
    const std::string key = tune_key(ctx, bvh, ap.nu * ap.nv, sw->max_bounces);
    if (tune_lookup(ctx, key, out)) return SBR_OK;
    void *dA;
    if ((rc = ctx->ws->get(W_TUNE, 64 * static_cast<size_t>(ns), &dA))) return rc;
    auto eval = [&](const sbr_tune &t, double *ms) -> int {
        sbr_sweep s2 = sub;
        s2.tune = &t;
        double best = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            sbr_stats st;
            int r = sbr_rcs_sweep(ctx, bvh, &s2, static_cast<double *>(dA), nullptr, &st);
            if (r) return r;
            if (rep > 0) best = std::min(best, st.ms_trace);  // the first run also warms caches
        }
        *ms = best;
        return SBR_OK;
    };
    sbr_tune cur = default_tune();
    double cur_ms;
    if ((rc = eval(cur, &cur_ms))) return rc;
    const int refills[] = {1, 16, 32, 48, 64};
    const int tiles[] = {4, 8, 16, 32};
    const int claims[] = {1, 2, 4, 8};
    const int blocks[] = {0, 2, 3};
    for (int pass = 0; pass < 4; ++pass) {
        const int *vals = pass == 0 ? refills : pass == 1 ? tiles : pass == 2 ? claims : blocks;
        const int nv = pass == 0 ? 5 : pass == 3 ? 3 : 4;
        for (int v = 0; v < nv; ++v) {
            sbr_tune t = cur;
            int &field = pass == 0 ? t.refill_min : pass == 1 ? t.tile_w : pass == 2 ? t.claim_tiles : t.blocks_per_cu;
            if (field == vals[v]) continue;
            field = vals[v];
            double ms;
            if ((rc = eval(t, &ms))) return rc;
            if (ms < cur_ms) {
                cur_ms = ms;
                cur = t;
            }
        }
    }
    tune_store(ctx, key, cur);
    *out = cur;
    return SBR_OK;
}
