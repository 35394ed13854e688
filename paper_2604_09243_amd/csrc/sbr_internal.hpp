// Internal declarations shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>
#include <climits>
#include <cstdint>
#include <cstddef>
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "../../include/sbr.h"

namespace sbr {

constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);
#define SBR_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::sbr::fail(SBR_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- device data
// BVH2 node: both child boxes inline (one 64-byte fetch tests two boxes).
//   a = (L.lo.x, L.lo.y, L.lo.z, L.hi.x)  b = (L.hi.y, L.hi.z, R.lo.x, R.lo.y)
//   c = (R.lo.z, R.hi.x, R.hi.y, R.hi.z)  ch = (left, right, -, -)
// child >= 0: internal node index; child < 0: leaf, ~child = first_slot * 8 +
// (count - 1): triangles [first_slot, first_slot + count) of the slot order.
struct __align__(16) BNode {
    float4 a, b, c;
    int4 ch;
};

// BVH4 node (128 bytes, one cache line): the boxes of up to four children,
// child i in component i of each float4 (lo.x of the four children, then
// hi.x, lo.y, hi.y, lo.z, hi.z), their references in ch (as in BNode: >= 0 an
// internal BVH4 node, < 0 a leaf code; kNoChild for an absent child, whose
// box repeats child 0's) and the child count in m.x.  Every box is a box of
// the BVH2 it is collapsed from (collapse_wide), so it holds the same
// guard-widened triangle boxes.
constexpr int kNoChild = INT32_MIN;
struct __align__(128) BNode4 {
    float4 lox, hix, loy, hiy, loz, hiz;
    int4 ch;
    int4 m;
};
static_assert(sizeof(BNode4) == 128, "a BVH4 node is one 128-byte line");

// Triangle in leaf (slot) order: p0 = (v0.xyz, input id as int bits),
// p1 = (e1.xyz, 0), p2 = (e2.xyz, 0).
struct __align__(16) BTri {
    float4 p0, p1, p2;
};

// Per-angle launch plan (device copy), built on the host in float64.
struct AnglePlan {
    double k[3], u[3], v[3];   // k = wave direction, u = phi_hat, v = theta_hat
    double uc, vc, s0, ds;
    float d32[3], eH32[3], eV32[3];
    int32_t nu, nv, tu, tv;    // rays, and tiles (tile_w x 64/tile_w rays) along u and v
    int64_t tile_base;         // first tile of this angle in the launch
    int64_t rec_base;          // first record slot of this angle
    int32_t root;              // root node of the angle's scene in the node array
    float eps;                 // the scene's surface offset
    float pbox;                // the scene's hit-rule box half-width P (SceneScale)
    // primary-ray mask: cells of kMaskCell x kMaskCell rays, rows of mcu bytes
    int32_t mcu;               // cells along u
    int64_t mask_base;         // first byte of this angle's cells in the launch's mask
    int64_t mwork_base;        // first build unit (one per node of the scene) of this angle
    int32_t node_cnt;          // nodes of the scene: [root, root + node_cnt)
    float mslack;              // margin of the projected leaf boxes, in ray spacings
};

// Primary-ray mask (silhouette of the leaf boxes, per angle): a ray whose
// cell no projected leaf box touches cannot pass a leaf's box test, so it is
// resolved as a miss without traversal.
constexpr int kMaskShift = 3;
constexpr int kMaskCell = 1 << kMaskShift;

// In-flight ray state of the wavefront schedule's queues, 6 x 16 bytes
// (structure of arrays): s0 = (o.xyz, tri_prev)  s1 = (d.xyz, tri_first)
// s2 = (eH.xyz, ray_id)  s3 = (eV.xyz, meta)  s4 = (P, comp)  s5 = (k.o0, -)
// meta = N | back << 7 | angle_slot << 8
struct RayQueue {
    float4 *s0, *s1, *s2, *s3;
    double2 *s4;
    double2 *s5;
};

// Hit record of one ray: one 64-byte block per slot, written whole by the
// lane whose ray ends (four 16-byte stores into one block, which the L2
// merges into full-sector writes; four arrays of 8-16 bytes per slot cost
// about twice the record bytes in partial-sector writes), read whole by PO.
//   r0 = (d_last.xyz, last hit: leaf slot, or triangle id in records packed
//   from caller hits)  r1 = (eH_last.xyz, tri_first)
//   r2 = (eV_last.xyz, N | flags << 8)  D = (D, 0)
struct __align__(64) Rec {
    float4 r0, r1, r2;
    double2 D;
};
static_assert(sizeof(Rec) == 64, "a record is one 64-byte block");
// held: one byte per record slot, 1 when slot e holds a record.  The slots
// of rays that never hit (or whose record was dropped) are neither written
// nor read; their byte stays 0.  The bytes are cleared (a kernel) before
// each launch that fills the records; every ray writes only its own byte,
// so no atomics are needed.
struct Records {
    Rec *rec;
    uint8_t *held;
};
// 32-bit words of a slot-byte array (cleared as words)
inline int64_t held_words(int64_t slots) { return (slots + 3) / 4; }

// Counter block, zeroed before each sweep chunk / trace call.  Counters that
// many waves update sit on separate 256-byte lines (kLineU32 uint32 apart):
//   stat:  u64[kStatU64] = [0] queries, [1] trapped, [8 + b] hits at bounce b,
//          [kStatMasked] primary rays resolved by the mask (counted in [0] too)
//   q_cnt: kQcnt lines; q_cnt[b] = rays pushed during bounce-b launch
//   claim: kMaxLaunch x kClaimRanges lines; the tile-claim counters of each
//          launch (kClaimRanges ranges, kClaimRanges / 8 per XCD)
constexpr int kLineU32 = 64;
constexpr int kClaimRanges = 64;
constexpr int kStatMasked = 8 + SBR_MAX_BOUNCES + 1;
constexpr int kStatU64 = kStatMasked + 1;
constexpr int kMaxLaunch = SBR_MAX_BOUNCES + 2;
constexpr int kQcnt = SBR_MAX_BOUNCES + 2;
constexpr size_t kStatBytes = 2048;
static_assert(8 * kStatU64 <= kStatBytes, "the stat counters fit their block");
constexpr size_t kCounterBytes = kStatBytes + 4ull * kLineU32 * (kQcnt + size_t(kClaimRanges) * kMaxLaunch);
struct CounterPtrs {
    unsigned long long *stat;
    uint32_t *q_cnt;
    uint32_t *claim;
};

constexpr int kScheduleStream = 0;
constexpr int kScheduleWavefront = 1;

struct Workspace;

// One scene of a multi-scene set (sbr_pack_scenes): where its nodes, leaf
// slots and triangle ids start in the set's arrays, and its geometry.
struct SceneInfo {
    int32_t root, slot_base, id_base, depth;
    int64_t n_tris, n_live, n_nodes;
    float eps;
    double diag;
    double bbox[6];
};

// Rounding scale of a scene.  M = X + C + 1.5 |diag| bounds the magnitude
// of every coordinate that the trace handles: X = the largest |coordinate| of
// the bounding box, C = the largest |coordinate| of its centre; the scene's
// points lie within X, and every origin of the aperture grid of any angle
// lies within `obound` = C + 1.5 |diag| (checked per plan by check_origins).
//   pbox:  the hit rule's box half-width P = fl32(2^-20 M): a float32 hit
//          point must lie in its triangle's box widened by P (the hit rule
//          of the float32 specification, the same on the oracle's side);
//   guard: G = fl32(2^-21 M), added around every widened triangle box in
//          the BVH, so that the float32 slab test of a node (its rounding,
//          and that of the hit point, are below 6 2^-24 M) never culls a
//          box that holds a hit point the rule accepts.
struct SceneScale {
    float pbox, guard;
    double obound;
};
inline SceneScale scene_scale(const double bbox[6], double diag)
{
    double X = 0.0, C = 0.0;
    for (int a = 0; a < 3; ++a) {
        X = std::max(X, std::max(std::fabs(bbox[a]), std::fabs(bbox[3 + a])));
        C = std::max(C, std::fabs(0.5 * (bbox[a] + bbox[3 + a])));
    }
    const double M = (X + C) + 1.5 * diag;
    SceneScale s;
    s.pbox = static_cast<float>(M * 0x1p-20);
    s.guard = static_cast<float>(M * 0x1p-21);
    s.obound = C + 1.5 * diag;
    return s;
}
// Box of triangle (v0, v0 + e1, v0 + e2) along one axis, widened by the hit
// rule's P (what the hit rule tests) and, for the BVH, by G as well.
__host__ __device__ inline void spec_box_axis(float v0, float e1, float e2, float P, float &lo, float &hi)
{
    const float p1 = v0 + e1, p2 = v0 + e2;
    lo = fminf(v0, fminf(p1, p2)) - P;
    hi = fmaxf(v0, fmaxf(p1, p2)) + P;
}

}  // namespace sbr

struct sbr_bvh {
    int device = 0;
    int leaf_size = 4;
    int64_t n_tris = 0, n_live = 0, n_nodes = 0;
    int32_t depth = 0;
    float eps = 0.f;
    double bbox[6] = {0, 0, 0, 0, 0, 0};
    double diag = 0.0;
    sbr::BNode *nodes = nullptr;  // [n_nodes]
    sbr::BNode4 *nodes4 = nullptr;  // [n_nodes4] the same tree collapsed to four children per node (NULL: none)
    int64_t n_nodes4 = 0;
    int32_t depth4 = 0;
    sbr::BTri *tris = nullptr;    // [n_live] in leaf order
    float4 *nrm_slot = nullptr;   // [n_live] unit normal in leaf order
    float4 *nrm_id = nullptr;     // [n_tris] unit normal by input index
    std::vector<float> host_normals;  // [n_tris*3]
    int64_t device_bytes = 0;
    std::vector<sbr::SceneInfo> scenes;  // a multi-scene set only (empty for one mesh)
    std::vector<std::pair<void *, size_t>> blocks;  // device blocks of the arrays above (block cache)
};

struct sbr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    sbr::Workspace *ws = nullptr;
    hipDeviceProp_t prop;
    std::map<std::string, sbr_tune> tune_cache;  // autotuned launch parameters
};

namespace sbr {

// Growable device scratch owned by a context.
struct Workspace {
    struct Buf {
        void *p = nullptr;
        size_t bytes = 0;
    };
    std::vector<Buf> bufs;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    ~Workspace();
    // Returns a device buffer of at least `bytes` for slot `i`; keeps it.
    int get(int i, size_t bytes, void **out);
    int get_pinned(size_t bytes, void **out);
};

// mesh_prep.cpp: host preparation of a float32 mesh (SBR_ERR_* status).
struct PreparedMesh {
    std::vector<float> v0, e1, e2, n;   // [nt*3] for every input triangle
    std::vector<uint8_t> degen;          // [nt]
    std::vector<int32_t> live;           // input ids of the non-degenerate triangles
    double bbox[6];
    double diag;
    float eps;
};
int prepare_mesh(const float *V, int64_t nv, const int32_t *T, int64_t nt, PreparedMesh &out);

// plan.cpp: frame and aperture of one angle (Eqs. L1-L3).
int plan_angle(const double bbox[6], double theta_deg, double phi_deg, double ds, double eta,
               sbr_angle_plan &out);

// lbvh.hip: builds nodes/tris on the device from a prepared mesh (linear
// BVH, or PLOC clustering over the same Morton order).
int build_lbvh(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh);
int build_ploc(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh);
// api.cpp: device memory of a BVH's arrays.  Blocks come from a per-device
// cache of blocks released by sbr_free_bvh (power-of-two size classes, at
// most 1 GiB held), so that repeated builds do not pay hipMalloc/hipFree.
int bvh_alloc(sbr_bvh *bvh, void **p, size_t bytes);
// A block of at least `bytes` of the cache (capacity in *cap), and its return;
// the caller guarantees that no work still uses a returned block.
int device_block_get(int device, size_t bytes, void **p, size_t *cap);
void device_block_put(int device, void *p, size_t cap);
// Host -> device copies on the context stream through its pinned staging
// buffer (the stream is synchronised before the buffer is refilled).
struct Upload {
    void *dst;
    const void *src;
    size_t bytes;
};
int upload_async(sbr_ctx *ctx, const std::vector<Upload> &ups);
// sah.cpp: the same node/triangle layout from a host binned-SAH build.
int build_sah(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh);
// sah.cpp: structural check of a node layout over n leaf slots (and, given
// the triangles in leaf order, of their ids in [0, n_ids) and leaf boxes).
int validate_layout(const std::vector<BNode> &hn, int n, int leaf_max, int depth, const std::vector<BTri> *tris,
                    int64_t n_ids, const SceneScale *scale);
// bvh4.cpp: collapses the BVH2 rooted at node 0 of hn into BVH4 nodes (root
// at 0, the four children of a node taken greedily by opening the child of
// largest surface area, sibling nodes stored together); depth4 = levels.
int collapse_wide(const std::vector<BNode> &hn, std::vector<BNode4> &out, int &depth4);
// bvh4.cpp: structural check of a BVH4 against the BVH2 it was collapsed from.
int validate_wide(const std::vector<BNode> &hn, const std::vector<BNode4> &w, int depth4);
// bvh4.cpp: builds bvh->nodes4 from bvh->nodes (a device -> host copy, the
// collapse on the host, an upload) unless it exists; SBR_OPT_BVH4 calls.
int build_wide(sbr_ctx *ctx, sbr_bvh *bvh);
// The wide copy for a call with these flags and schedule: built on first use
// (the copy is a cache of the tree, hence the cast).
inline int ensure_wide(sbr_ctx *ctx, const sbr_bvh *bvh, uint32_t flags, int schedule)
{
    if (!(flags & SBR_OPT_BVH4) || bvh->nodes4 || !bvh->scenes.empty() || schedule != kScheduleStream) return 0;
    return build_wide(ctx, const_cast<sbr_bvh *>(bvh));
}
// Traversal stack entries the tree needs: BVH2 one per level, BVH4 three.
inline int stack_need(const sbr_bvh *bvh, bool wide) { return wide ? 3 * bvh->depth4 + 1 : bvh->depth; }
// sah.cpp: surface-area estimates of the traversal work of a node layout.
void layout_quality(const std::vector<BNode> &hn, sbr_bvh_quality &q);

// trace.hip
struct TraceArgs {
    const sbr_bvh *bvh;
    int bmax;
    uint32_t flags;
    int schedule;             // kScheduleStream or kScheduleWavefront
    int tile_shift;           // log2 of the tile width
    int claim_tiles, refill_min, blocks;
    // grid source (sweep)
    const AnglePlan *plans;   // device [n_angles]
    const int64_t *tile_base; // device [n_angles + 1]
    int n_angles;
    int64_t n_tiles;
    const uint8_t *mask;      // device primary-ray mask of the plans, or NULL (every ray traced)
    const int32_t *live;      // streaming schedule: live tiles of the mask (launch_live), or NULL
    const uint32_t *live_count;
    // user source / sink (sbr_trace)
    const sbr_rays *rays;
    int64_t n_rays;
    const sbr_hits *hits;
    double k_hat[3];
    // queues (wavefront schedule), records (sweep), counters
    RayQueue q_in, q_out;
    Records rec;
    CounterPtrs ctrs;
    int32_t *spill;           // device traversal-stack spill
};
// bounce = 1 for the stream schedule (one launch does every bounce)
int launch_trace(hipStream_t s, const TraceArgs &a, int bounce);
// The live tiles of a masked launch (at least one non-empty mask cell), in
// tile order, into live[0, *count); the in-grid positions of the other tiles
// are added to the masked and query statistics.  blk holds
// live_blocks(n_tiles) + 1 words, the last of them the count.
int64_t live_blocks(int64_t n_tiles);
int launch_live(hipStream_t s, const TraceArgs &a, int32_t *live, uint32_t *blk);
// Static scratch of the no-alloc trace (one per device, kNoallocScratchBytes):
// noalloc_scratch_setup looks up this device's address (the device must be
// current; done once by sbr_create); noalloc_counters lays the counter block
// of one streaming launch over it (base and the bytes to clear).
constexpr size_t kNoallocScratchBytes = 40960;
int noalloc_scratch_setup(int device);
int noalloc_counters(int device, CounterPtrs &c, void **base, size_t *bytes);
// Builds the primary-ray mask of plans [0, n_angles) of one launch: zeroes
// mask[0, mask_bytes) (a kernel, so usable inside a captured graph), then
// marks every cell that the padded projection of a leaf box of the angle's
// scene touches; n_units = sum of the plans' node_cnt.
int launch_mask(hipStream_t s, const BNode *nodes, const AnglePlan *plans, int n_angles, int64_t n_units,
                uint8_t *mask, int64_t mask_bytes);
// Host: margins and cell rows of a plan for the mask (scene bbox, node count)
void mask_plan(AnglePlan &p, const double bbox[6], int64_t node_cnt);
// Ties plan p to its scene (root node, eps, the hit rule's P, the mask's
// margin) and checks that every origin of its ray grid lies within the
// scene's `obound` (SceneScale); SBR_ERR_SAMPLING otherwise (a spacing
// coarser than a fifth of the scene's diagonal).
int scene_plan(AnglePlan &p, int32_t root, float eps, const double bbox[6], double diag, int64_t node_cnt);
// Host: mask_base / mwork_base of plans [a0, a1) of one launch; returns the
// launch's mask bytes (a multiple of 4) and build units.
void mask_layout(AnglePlan *plans, int64_t a0, int64_t a1, int64_t &bytes, int64_t &units);
int trace_persistent_blocks(sbr_ctx *ctx, int blocks_per_cu);  // 0 = occupancy limit
int check_tune(const sbr_tune &t);
int trace_block_threads();
int trace_stack_lds();  // LDS entries of the stack when it spills
bool trace_needs_spill(const sbr_bvh *bvh, bool wide);
// Whether a launch over this tree walks its BVH4 copy (SBR_OPT_BVH4 on the
// streaming schedule of a one-mesh tree whose copy exists).
bool trace_walks_wide(const sbr_bvh *bvh, uint32_t flags, int schedule);

// api.cpp helpers shared with the batch entry points
sbr_tune default_tune();
int normalize_tune(sbr_tune &t);           // check_tune, then chunk_log2 0 -> default
// Automatic chunk size (chunk_log2 0) of a sweep or batch, on the current
// device: 2^30 rays when their record slots (64 bytes and a slot byte each,
// 69 GB) fit in a quarter of the device memory that is free or already held
// (held_bytes: the caller's own record buffers, about to be replaced), else
// kDefaultChunkLog2.  The chunking changes no result (each chunk is traced
// and summed the same way); larger chunks mean fewer launch tails.
int auto_chunk_log2(size_t held_bytes);
// claim_tiles 0 (automatic): one tile per claim when the tree outgrows an
// XCD's L2 (waves on neighbouring tiles at once then share its node and
// triangle lines), two otherwise (fewer claims of cheap tiles)
constexpr int64_t kL2BytesPerXcd = int64_t(4) << 20;
int auto_claim_tiles(const sbr_bvh *bvh);
int log2i(int x);
void fill_stats(sbr_stats *st, const unsigned long long *hstat, int bmax, int64_t rays, bool drop_trapped,
                int64_t chunks);
// Every bounce of one trace (one streaming launch, or one launch per bounce
// with the queues swapped); ev (nullable) gets an event after each launch.
int run_trace(hipStream_t s, TraceArgs &a, RayQueue qa, RayQueue qb, std::vector<hipEvent_t> *ev);
size_t spill_words(const sbr_bvh *bvh, int blocks);
// Device plan of one angle from its host plan (tiles of tile_w x 64/tile_w).
void fill_plan(const sbr_angle_plan &ap, double ds, int tile_w, AnglePlan &p);
// Rays per chunk by default: 2^29 for sweeps and batches.  A chunk's records
// (64 bytes per ray: 34 GB at 2^29) stay on the device between its trace and
// its PO; larger chunks mean fewer launches and fewer launch tails (the
// 64-scene batch replays in 2.18 / 1.89 / 1.82 s with 2^26 / 2^28 / 2^29-ray
// chunks, the aircraft sweep traces in 233 / 200 / 194 ms; 2^30 gains 2 %
// more for 69 GB, taken where the device has room: auto_chunk_log2).
constexpr int kDefaultChunkLog2 = 29;
// Autotuner cache: the context's map, then the JSON-lines file named by
// $SBR_TUNE_CACHE (if any).
bool tune_lookup(sbr_ctx *ctx, const std::string &key, sbr_tune *out);
void tune_store(sbr_ctx *ctx, const std::string &key, const sbr_tune &t);
int size_bucket(double x);  // floor(log2(x)), 0 below 1

// po.hip
// One incidence angle of a PO launch (device copy, built on the host).
struct PoAngle {
    double basis[9];            // k_hat, theta_hat, phi_hat
    double dA;                  // ray-tube area (ray spacing squared)
    int64_t rec_base, rec_cnt;  // record slots [rec_base, rec_base + rec_cnt)
    int64_t unit_base;          // first PO block of the angle in the launch
    int64_t part_base;          // first partial row (8 int64) of the angle
    int64_t out_base;           // output row of the angle's first frequency
    int32_t kf_off, n_f;        // its wavenumbers kf[kf_off, kf_off + n_f)
    double dk;                  // their spacing if evenly spaced, else 0
};
// Spacing of n wavenumbers if they form an arithmetic progression (to a few
// ulps), else 0.
double uniform_step(const double *kf, int n);
struct PoArgs {
    const sbr_bvh *bvh;
    Records rec;
    const PoAngle *ang;  // device [n_angles]
    int n_angles;
    int64_t n_units;     // blocks of the launch: sum over angles of ceil(rec_cnt / kPoRecsPerBlock)
    int max_nf;          // largest n_f of the angles
    int mode;
    const double *kf;    // device wavenumbers
    long long *partial;  // device partial rows
    int fp32;            // SBR_OPT_FP32_PATH: the phase k D in float32 (precision study)
    int rec_slots;       // the records' last triangle is a leaf slot (trace records), else an input id
    int kinds;           // kPoEven | kPoUneven: which spacings the angles have (0: not known, both)
};
// Angle kinds of a PO launch: evenly spaced wavenumbers (dk != 0), or not
// (dk == 0, one frequency included); each has its own many-frequency kernel.
constexpr int kPoEven = 1, kPoUneven = 2;
inline int po_kind(double dk) { return dk != 0.0 ? kPoEven : kPoUneven; }
constexpr int kPoRecsPerBlock = 4096;
__host__ __device__ inline int64_t po_units(int64_t rec_cnt) { return (rec_cnt + kPoRecsPerBlock - 1) / kPoRecsPerBlock; }
int launch_po(hipStream_t s, const PoArgs &a);
// A_out rows (8 doubles) and sigma rows (4 doubles) are indexed by out_base + f.
int launch_po_finalize(hipStream_t s, const PoArgs &a, double *A_out, double *sigma_out);
// Converts caller hit arrays into n record slots (invalid rays keep no flags).
int launch_pack_hits(hipStream_t s, const sbr_hits *h, int64_t n, Records rec);

// scene.hip
// Fills n uint32 words with zero (usable inside a captured graph).
int launch_zero_u32(hipStream_t s, uint32_t *p, int64_t n);
// Relocation of one scene's nodes and triangles into a multi-scene arena.
int launch_relocate(hipStream_t s, const BNode *src_nodes, int64_t n_nodes, BNode *dst_nodes, int32_t node_off,
                    const BTri *src_tris, int64_t n_slots, BTri *dst_tris, int32_t slot_off, int32_t id_off);

// mlp.hip: surrogate network kernels
constexpr int kActSilu = 0, kActRelu = 1;
constexpr int kEpiHidden = 0, kEpiDz = 1, kEpiF32 = 2;
// C[m][n] = sum_k A[m][k] B[n][k] (bf16, fp32 accumulation); M % 64 == 0,
// N % 128 == 0, K % 16 == 0.  Epilogues:
//   kEpiHidden: z = C + bias[n] (zout, optional), h = bf16(act(z)) to hout
//               and, optional, to htout transposed
//   kEpiDz:     dz = C act'(zin) to fout, bf16(dz) to hout and htout (transposed)
//   kEpiF32:    C to fout
struct GemmArgs {
    const uint16_t *A;
    int64_t lda;
    const uint16_t *B;
    int64_t ldb;
    int M, N, K;
    const float *bias;
    int act;
    float *zout;
    int64_t ldz;
    uint16_t *hout;
    int64_t ldh;
    uint16_t *htout;
    int64_t ldht;
    const float *zin;
    int64_t ldzi;
    float *fout;
    int64_t ldf;
    int ksplit = 1;           // kEpiF32 only: K split over blockIdx.z ...
    int64_t split_stride = 0; // ... into fout slices this many floats apart
};
struct MlpNorm {
    double lo[3], hi[3];
};
int launch_gemm(hipStream_t s, int epi, const GemmArgs &g);
int launch_embed(hipStream_t s, const double *pts, int64_t M, int64_t Mpad, const MlpNorm &nm, const float *Bff,
                 int n_ff, uint16_t *h0, uint16_t *h0t);
int launch_out(hipStream_t s, const uint16_t *h, int width, const uint16_t *wo, const float *bo, int64_t M,
               int64_t Mrows, int mode, double scale, double *A, const float *tgt, float *dy, float *partial);
constexpr int kMaxLayers = 9;
struct RefreshTable {
    const float *w;
    uint16_t *wb, *wt;
    uint16_t *wf;  // fragment-major copies (layers with frag[l] != 0), at woff[l]
    int n_layers;
    int rows[kMaxLayers], cols[kMaxLayers], frag[kMaxLayers];
    int64_t woff[kMaxLayers], toff[kMaxLayers];
};
int launch_refresh(hipStream_t s, const RefreshTable &t);
// Training batch rows idx[0, count) of the points and targets, their Fourier
// features (h0 and its transpose) and targets / out_scale; *bump (nullable)
// += 1, the device step count of a training step.
int launch_embed_batch(hipStream_t s, const double *pts, const double *tc, const int32_t *idx, int64_t count,
                       int64_t Mpad, const MlpNorm &nm, const float *Bff, int n_ff, double inv_scale, uint16_t *h0,
                       uint16_t *h0t, float *tb, int64_t *bump);
// The output layer's backward pass: the last hidden layer's gradient (dz,
// bf16 dz and its transpose), the output weight and bias gradients (gw, gb)
// and the batch loss (*loss = sum of part[0, n_part)).
struct OutBackIn {
    const float *dy;
    const uint16_t *wo;
    int width;
    int64_t Mrows;
    const float *z;
    int act;
    float *dz;
    uint16_t *dzb, *dzbt;
    const uint16_t *h;
    const float *part;
    int n_part;
    float *loss;
};
struct OutBackArgs : OutBackIn {
    float *pw, *pb;  // weight and bias partials per 64-row group
    int64_t nb_back;
    int gx, R;
};
struct SumJob {
    const float *part;
    int nz;
    int64_t n;
    float *out;
};
struct ColsumArgs {
    const float *x;
    int64_t rows;
    int cols;
    float *part;
    int gx, R;
};
// Two slice sums (out[i] = sum over z of part[z][i]) and their block counts
// (64 outputs per block; a count of 0: no sum).
struct SumPair {
    SumJob a, b;
    int64_t nba, nbb;
};
// The gradient sums a launch leaves pending are run as extra blocks of the
// next launch that reads none of their buffers (launch_wgrad_colsum,
// launch_gemm_fold) or on their own (launch_sum_pair).
// scratch: at least ceil(Mrows / 64) (4 width + 4) floats; *pending: the
// output layer's weight and bias gradient sums.
int launch_out_backward(hipStream_t s, const OutBackIn &in, float *gw, float *gb, float *scratch, SumPair *pending);
// A hidden layer's weight gradient (split-K product g into its float32
// slices g.fout) and the column-sum partials of its bias gradient (the
// layer's output gradient dz [rows][cols] into colpart, at least
// ceil(rows / 64) cols floats), plus the pending sums `fold`; *pending: the
// sums into gw and gb.
int launch_wgrad_colsum(hipStream_t s, const GemmArgs &g, const float *dz, int64_t rows, int cols, float *colpart,
                        float *gw, float *gb, const SumPair &fold, SumPair *pending);
// A product (launch_gemm, no k split, kEpiHidden or kEpiDz) plus the pending sums `fold`.
int launch_gemm_fold(hipStream_t s, int epi, const GemmArgs &g, const SumPair &fold);
int launch_sum_pair(hipStream_t s, const SumPair &p);
// Adam over n parameters at step *step - 1 (the step count is advanced at
// the start of each training step) with lr_sched[*step - 1 - step0], then
// the bf16 copies of the updated weights (rt, as launch_refresh).
int launch_adam(hipStream_t s, float *w, float *m, float *v, const float *g, int64_t n, const float *lr_sched,
                const int64_t *step, int64_t step0, float b1, float b2, float eps, const RefreshTable &rt);
// Whole-network inference for width 256 (activations in LDS).
struct FusedArgs {
    const double *pts;
    int64_t M;
    MlpNorm norm;
    const float *Bff;
    int n_ff, depth, act;
    const uint16_t *wf[kMaxLayers];  // hidden layer weights, bf16 [256][n_in], fragment-major
    const float *b[kMaxLayers];
    const uint16_t *wo;             // output layer bf16 [4][256]
    const float *bo;
    double scale;
    double *A;                      // [M][4]
};
bool fused_ok(int n_ff, int width, int depth);
int launch_mlp_fused(hipStream_t s, const FusedArgs &f);
int launch_grid_pts(hipStream_t s, const double *th, const double *ph, const double *fr, int64_t na, int nf,
                    double *pts);
int launch_probe_check(hipStream_t s, const double *A_sbr, const double *A_sur, int64_t n_ta, int n_tf, int per_tile,
                       double *smax, double floor_db, double tol_db, uint8_t *flag, double *err);
int launch_scatter_copol(hipStream_t s, const double *A, const int64_t *dst, int64_t n, double *out);

}  // namespace sbr
