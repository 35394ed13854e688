// Internal declarations shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
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
};

// In-flight ray state of the wavefront schedule's queues, 6 x 16 bytes
// (structure of arrays): s0 = (o.xyz, tri_prev)  s1 = (d.xyz, tri_first)
// s2 = (eH.xyz, ray_id)  s3 = (eV.xyz, meta)  s4 = (P, comp)  s5 = (k.o0, -)
// meta = N | back << 7 | angle_slot << 8
struct RayQueue {
    float4 *s0, *s1, *s2, *s3;
    double2 *s4;
    double2 *s5;
};

// Hit record of one ray (structure of arrays); r2.w carries N | flags << 8,
// zero for a ray that never hit.
//   r0 = (d_last.xyz, tri_last)  r1 = (eH_last.xyz, tri_first)
//   r2 = (eV_last.xyz, N | flags << 8)  D
struct Records {
    float4 *r0, *r1, *r2;
    double *D;
};

// Counter block, zeroed before each sweep chunk / trace call.  Counters that
// many waves update sit on separate 256-byte lines (kLineU32 uint32 apart):
//   stat:  u64[kStatU64] = [0] queries, [1] trapped, [8 + b] hits at bounce b
//   q_cnt: kQcnt lines; q_cnt[b] = rays pushed during bounce-b launch
//   claim: kMaxLaunch x 8 lines; the 8 tile-claim counters of each launch
constexpr int kLineU32 = 64;
constexpr int kStatU64 = 8 + SBR_MAX_BOUNCES + 1;
constexpr int kMaxLaunch = SBR_MAX_BOUNCES + 2;
constexpr int kQcnt = SBR_MAX_BOUNCES + 2;
constexpr size_t kStatBytes = 1024;
constexpr size_t kCounterBytes = kStatBytes + 4ull * kLineU32 * (kQcnt + 8 * kMaxLaunch);
struct CounterPtrs {
    unsigned long long *stat;
    uint32_t *q_cnt;
    uint32_t *claim;
};

constexpr int kScheduleStream = 0;
constexpr int kScheduleWavefront = 1;

struct Workspace;

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
    sbr::BTri *tris = nullptr;    // [n_live] in leaf order
    float4 *nrm_slot = nullptr;   // [n_live] unit normal in leaf order
    float4 *nrm_id = nullptr;     // [n_tris] unit normal by input index
    std::vector<float> host_normals;  // [n_tris*3]
    int64_t device_bytes = 0;
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

// lbvh.hip: builds nodes/tris on the device from a prepared mesh.
int build_lbvh(sbr_ctx *ctx, const PreparedMesh &pm, int leaf_max, sbr_bvh *bvh);

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
int trace_persistent_blocks(sbr_ctx *ctx, int blocks_per_cu);  // 0 = occupancy limit
int check_tune(const sbr_tune &t);
int trace_block_threads();
int trace_stack_lds();  // LDS entries of the stack when it spills
bool trace_needs_spill(const sbr_bvh *bvh);

// po.hip
struct PoArgs {
    const sbr_bvh *bvh;
    Records rec;
    const uint32_t *rec_cnt;  // [n_angles * cnt_stride]: record slots of each angle
    int cnt_stride;
    const int64_t *rec_base;  // [n_angles]: first record slot of each angle
    int n_angles;
    int chunks;               // blocks per angle along x
    int mode;
    const double *kf;         // device [n_freq] wavenumbers
    int n_freq;
    const double *basis;      // device [n_angles][9]: k, theta_hat, phi_hat
    long long *partial;       // device [n_angles][chunks][n_freq][8]
};
constexpr int kPoRecsPerBlock = 4096;
int launch_po(hipStream_t s, const PoArgs &a);
int launch_po_finalize(hipStream_t s, const PoArgs &a, double dA, double *A_out, double *sigma_out);
int launch_pack_hits(hipStream_t s, const sbr_hits *h, int64_t n, Records rec, uint32_t *cnt);

}  // namespace sbr
