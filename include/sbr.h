/*
 * sbr.h -- C ABI of the MI355X (gfx950) SBR trace-integrate library.
 *
 * The library computes the monostatic radar cross section of a perfectly
 * conducting triangle mesh by shooting and bouncing rays (arXiv 2604.09243):
 * an orthographic ray grid per incidence angle (Sec. 4, Eqs. L1-L3), multi-
 * bounce specular transport through a BVH (Algorithm 2), and the ray-tube
 * physical-optics sum over the valid hits (Eq. po_sum; Eqs. em5-em6), giving
 * sigma = 4 pi |A|^2 (Sec. 4, trace-integrate paragraph).
 *
 * Conventions (all entry points):
 *  - Every call returns an sbr_status; on a non-OK status a message is
 *    available from sbr_last_error() (thread-local, valid until the next
 *    failing call on the same thread).  No call throws across the ABI.
 *  - Inputs are borrowed; the library never frees caller memory.  Output
 *    buffers are caller-owned and must be large enough for the documented
 *    shape.  "device" pointers are HIP device (or managed) memory on the
 *    context's device; "host" pointers are ordinary host memory.
 *  - Device work is enqueued on the context stream and is asynchronous
 *    unless the SBR_OPT_SYNC flag is given; results in device buffers are
 *    valid after the stream has been synchronised.  Statistics structs
 *    (host) are filled only when the call synchronises (SBR_OPT_SYNC, or a
 *    non-NULL stats pointer, which implies a synchronisation).
 *  - Option structs begin with struct_size (set it to sizeof the struct).
 *  - Units: metres, hertz, degrees at the API.  Polarisation index 0 = H
 *    (phi_hat), 1 = V (theta_hat).  Complex values are two doubles (re, im).
 *  - Angles: theta is the polar angle from +z, phi the azimuth; the radar
 *    sits along r = (sin t cos p, sin t sin p, cos t) and the incident wave
 *    travels along k = -r.
 */
#ifndef SBR_H
#define SBR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBR_ABI_VERSION 2
#define SBR_MAX_BOUNCES 127

typedef struct sbr_ctx sbr_ctx; /* device + stream + workspace */
typedef struct sbr_bvh sbr_bvh; /* prepared mesh + BVH in device memory */

typedef enum {
    SBR_OK = 0,
    SBR_ERR_INVALID_ARG = -1,  /* bad pointer, size, enum or option */
    SBR_ERR_INVALID_MESH = -2, /* non-finite vertex or index out of range */
    SBR_ERR_SAMPLING = -3,     /* ray spacing coarser than lambda/5 */
    SBR_ERR_OOM = -4,          /* device or host allocation failed */
    SBR_ERR_HIP = -5,          /* HIP runtime error (message has details) */
    SBR_ERR_OVERFLOW = -6,     /* a count exceeds a documented limit */
    SBR_ERR_UNSUPPORTED = -7   /* feature not available on this device */
} sbr_status;

enum { SBR_POL_H = 0, SBR_POL_V = 1 };

/* PO sum (Eq. po_sum and its polarimetric reading):
 *  SBR_MODE_VECTOR: Eqs. em5-em6 applied to each ray tube's footprint on
 *    its last facet, with the field reflected at every PEC hit; gives all
 *    four (receive, transmit) polarisation pairs.
 *  SBR_MODE_PAPER:  Eq. po_sum literally (first-hit obliquity, Gamma = -1);
 *    co-polar only (HH = VV, cross-polar terms are zero). */
enum { SBR_MODE_VECTOR = 0, SBR_MODE_PAPER = 1 };

enum { SBR_MEM_HOST = 0, SBR_MEM_DEVICE = 1 };

/* per-ray record flags (sbr_hits.flags) */
#define SBR_REC_VALID 1     /* at least one hit (Algorithm 2 "valid") and not dropped */
#define SBR_REC_TRAPPED 2   /* still hitting after max_bounces (see SBR_OPT_DROP_TRAPPED) */
#define SBR_REC_BACK_LAST 4 /* the last hit was on the side opposite the stored normal */

/* option flags (sbr_trace_opts.flags, sbr_sweep.flags) */
#define SBR_OPT_DROP_TRAPPED 1        /* one extra query at max_bounces; rays that hit are invalid */
#define SBR_OPT_PAPER_PATH 2          /* path = sum of t only (no offset correction) */
#define SBR_OPT_ALLOW_UNDERSAMPLING 4 /* accept ray spacing coarser than lambda/5 */
#define SBR_OPT_SYNC 8                /* synchronise the stream before returning */
#define SBR_OPT_WAVEFRONT 16          /* one launch per bounce with a compacted ray queue between
                                         launches (default: one streaming launch for all bounces) */
#define SBR_OPT_NO_GRAPH 32           /* sbr_batch_run: launch eagerly instead of replaying the
                                         captured graph (gives per-stage times in sbr_stats) */
#define SBR_OPT_NO_MASK 64            /* sweeps and batches: trace every primary ray.  By default a
                                         per-angle mask of 8 x 8-ray cells, built on the device from
                                         the projected leaf boxes of the tree (with a margin above
                                         the box test's float32 rounding), resolves rays of empty
                                         cells as misses without traversal; results are identical */
#define SBR_OPT_FP32_PATH 128         /* precision study of Sec. 6, not the method: the path P, the
                                         distance D and the phase k D in float32 instead of float64
                                         (sbr_trace and sbr_rcs_sweep; batches refuse it) */
#define SBR_OPT_FP64_TRAVERSE 256     /* precision and timing study of Sec. 6 (its single vs double
                                         precision trace times), not the method: box and
                                         triangle tests in float64 (hits then differ from the
                                         float32 specification by rounding); streaming schedule
                                         of sbr_trace and sbr_rcs_sweep only */
#define SBR_OPT_PACKET 1024           /* traversal study, sweeps and batches: the parallel primary
                                         rays of a tile walk the tree together (one shared stack,
                                         every node and triangle read once per wave) instead of each
                                         on its own; results are identical either way */
#define SBR_OPT_BVH4 512              /* traversal study: walk a four-wide copy of the tree
                                         (four child boxes per 128-byte node, collapsed from the
                                         binary tree on the host at the first such call and kept
                                         with the BVH) instead of the binary tree.  The same
                                         results bit for bit; measured slower on the aircraft,
                                         so not the default.  sbr_trace and sbr_rcs_sweep on the
                                         streaming schedule; sbr_trace_noalloc refuses it */

/* ------------------------------------------------------------------------ */
/* Library and context                                                       */
/* ------------------------------------------------------------------------ */

/* SBR_ABI_VERSION of the built library. */
int sbr_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *sbr_last_error(void);

/* Creates a context on HIP device `device` enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * context, released with sbr_destroy.  Errors: INVALID_ARG (no device of
 * that index, NULL out), HIP. */
int sbr_create(sbr_ctx **out, int device, void *hip_stream);

/* Changes the stream later calls enqueue on. */
int sbr_set_stream(sbr_ctx *ctx, void *hip_stream);

/* Blocks until all work enqueued by the context has finished. */
int sbr_synchronize(sbr_ctx *ctx);

/* Frees the context and its workspace.  BVHs built with it must be freed
 * first.  NULL is accepted. */
void sbr_destroy(sbr_ctx *ctx);

/* ------------------------------------------------------------------------ */
/* sbr_build_bvh -- mesh preparation and BVH (Sec. 4 BVH paragraph; the      */
/* paper's host-built Algorithm 1 is replaced by a GPU LBVH)                 */
/* ------------------------------------------------------------------------ */

enum { SBR_BUILD_LBVH = 0, SBR_BUILD_SAH = 1, SBR_BUILD_PLOC = 2 };

typedef struct {
    uint32_t struct_size;
    int32_t mem;       /* SBR_MEM_HOST or SBR_MEM_DEVICE: where verts/tris live */
    int32_t leaf_size; /* triangles per leaf, 1..4 (subtrees that small become leaves); 0 = 4 */
    int32_t builder;   /* SBR_BUILD_LBVH: Morton-code LBVH on the GPU (default);
                          SBR_BUILD_SAH: binned surface-area-heuristic build on the host (Algorithm 1
                          with its SAH cost), slower to build, fewer node and triangle tests per ray;
                          SBR_BUILD_PLOC: on the GPU, agglomerative clustering of the LBVH's Morton
                          order by merged surface area, leaves chosen by the SAH cost: a tree of
                          the host SAH build's quality at GPU build speed */
} sbr_bvh_opts;

typedef struct {
    int64_t n_tris;       /* triangles given */
    int64_t n_live;       /* non-degenerate triangles (in the BVH) */
    int64_t n_nodes;      /* internal nodes of the layout (at most n_live - 1, at least 1) */
    int32_t depth;        /* longest root-to-leaf path (edges) */
    float eps;            /* surface offset (1e-5 of the bounding-box diagonal) */
    double bbox[6];       /* lo xyz, hi xyz of the referenced vertices */
    int64_t device_bytes; /* device memory held by the BVH */
    int32_t n_scenes;     /* 1, or the scene count of a set made by sbr_pack_scenes */
    int32_t reserved;
} sbr_bvh_info;

/* verts: [n_verts][3] float32 (metres); tris: [n_tris][3] int32 vertex
 * indices; both in host or device memory per opts->mem (NULL opts = host).
 * Copies what it needs into library-owned device memory; *out is released
 * by sbr_free_bvh.  Per triangle: e1 = v1 - v0, e2 = v2 - v0 (float32), unit
 * normal from e1 x e2 evaluated in float64; triangles with area below
 * 1e-12 * diag^2 are degenerate and skipped (not an error).  Errors:
 * INVALID_MESH (non-finite vertex, index outside [0, n_verts)),
 * INVALID_ARG (n_tris < 1 or > 2^28, NULL pointers), OOM, HIP.  Blocks the
 * host until the BVH is complete. */
int sbr_build_bvh(sbr_ctx *ctx, const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                  const sbr_bvh_opts *opts, sbr_bvh **out);

int sbr_bvh_get_info(const sbr_bvh *bvh, sbr_bvh_info *out);

/* Checks the layout of a one-mesh BVH (any builder) on the host: every node
 * reachable once from the root in preorder, child boxes inside their
 * parent's box, every leaf slot in exactly one leaf of at most leaf_size
 * triangles, every triangle's corners inside the box its leaf is reached
 * through, every input id in at most one slot, the depth bound kept; and
 * the four-wide copy of SBR_OPT_BVH4 once it exists: every BVH2 leaf
 * reached exactly once with the box the BVH2 gives it, child boxes inside
 * their parent's, the child counts and its depth bound.
 * Copies the arrays to the host (synchronous).  Errors: INVALID_MESH with
 * the first violation, UNSUPPORTED for a scene set, INVALID_ARG, HIP. */
int sbr_bvh_validate(const sbr_bvh *bvh);

/* Surface-area estimates of a layout's traversal work (the cost model of
 * the SAH build, Sec. 4): for straight lines that meet the root box, a node
 * is reached with probability area(node box) / area(root box).  Lets
 * callers compare trees of different builders without tracing. */
typedef struct {
    double node_visits; /* expected internal-node visits (each tests two child boxes) */
    double tri_tests;   /* expected triangle tests */
    int64_t leaves;     /* leaf references */
    int64_t leaf_tris;  /* triangles over all leaves */
    int32_t max_depth;  /* internal nodes on the longest root-to-leaf path */
    int32_t reserved;
} sbr_bvh_quality;

/* One-mesh BVH only (UNSUPPORTED for a scene set); copies the nodes to the
 * host (synchronous).  Errors: INVALID_ARG, UNSUPPORTED, HIP. */
int sbr_bvh_quality_of(const sbr_bvh *bvh, sbr_bvh_quality *out);

/* Unit normals of all n_tris triangles in input order ([n_tris][3] float32,
 * host memory; zero for degenerate triangles). */
int sbr_bvh_normals(const sbr_bvh *bvh, float *out_host);

void sbr_free_bvh(sbr_bvh *bvh);

/* ------------------------------------------------------------------------ */
/* sbr_trace -- multi-bounce transport of caller rays (Algorithm 2)          */
/* ------------------------------------------------------------------------ */

/* Rays, device memory, [n][3] float32 each.  eH/eV: transmit polarisation
 * vectors carried with each ray (unit, orthogonal to d). */
typedef struct {
    const float *o;
    const float *d;
    const float *eH;
    const float *eV;
} sbr_rays;

/* Per-ray results, device memory, caller-allocated, indexed by ray.  Any
 * pointer may be NULL to skip that output.  "last" quantities are those
 * arriving at the last hit (before its reflection). */
typedef struct {
    int32_t *n_bounce;  /* [n] number of hits N (0 = missed) */
    int32_t *tri_first; /* [n] input index of the first triangle hit, -1 if none */
    int32_t *tri_last;  /* [n] input index of the last triangle hit, -1 if none */
    int32_t *flags;     /* [n] SBR_REC_* */
    double *path;       /* [n] one-way path P along the ray (float64) */
    double *D;          /* [n] round-trip phase path k.o + P + k.x_last (float64) */
    float *d_last;      /* [n][3] */
    float *x_last;      /* [n][3] */
    float *eH_last;     /* [n][3] */
    float *eV_last;     /* [n][3] */
    int32_t *tri_path;  /* [n][max_bounces] triangle hit at each bounce, -1 after the end */
} sbr_hits;

typedef struct {
    uint32_t struct_size;
    uint32_t flags;  /* SBR_OPT_DROP_TRAPPED | SBR_OPT_PAPER_PATH | SBR_OPT_SYNC */
    double k_hat[3]; /* direction defining D (usually the launch direction) */
} sbr_trace_opts;

typedef struct {
    int64_t rays;      /* rays launched */
    int64_t queries;   /* closest-hit queries (rays x bounces incl. the final miss) */
    int64_t valid;     /* rays with SBR_REC_VALID */
    int64_t trapped;   /* rays with SBR_REC_TRAPPED */
    int64_t hits[SBR_MAX_BOUNCES + 1]; /* hits[b] = rays that hit at bounce b (1-based) */
    int64_t angles;    /* incidence angles processed */
    double ms_trace;   /* GPU time of ray generation + all bounces */
    double ms_po;      /* GPU time of the PO sum + finalize */
    double ms_total;   /* wall time of the call */
    double ms_bounce[SBR_MAX_BOUNCES + 1];       /* GPU time of the bounce-b launches (1-based;
                                                    SBR_OPT_WAVEFRONT only) */
    int64_t queries_bounce[SBR_MAX_BOUNCES + 1]; /* queries made by the bounce-b launches */
    int64_t trav[6]; /* libraries built with SBR_TRACE_COUNTERS only (else 0): node visits, leaf
                        visits, triangle tests (summed over queries), and wave-level trips of the
                        node loop, the leaf step and the bounce loop */
    int64_t masked;  /* primary rays resolved as misses by the mask (included in queries) */
    int64_t chunks;  /* trace launches of the streaming schedule (one per chunk of angles or items) */
} sbr_stats;

/* Traces n_rays rays (1 <= n_rays < 2^31) for up to max_bounces (1..SBR_MAX_BOUNCES)
 * reflections (Algorithm 2, Sec. 4).  A triangle is hit when the float32
 * Moller-Trumbore test accepts it (u >= 0, v >= 0, u + v <= 1, 0 < t) and
 * the float32 hit point o + t d lies in the triangle's axis-aligned box
 * widened by P = fl32(2^-20 M) on every side, with M = X + C + 1.5 |diag|
 * (X: largest |coordinate| of the mesh's bounding box, C: that of its
 * centre); the second condition refuses only hits whose float32 point has
 * drifted off the triangle (slivers seen from afar, grazing rays).  Closest
 * hit = smallest (t, input triangle index) over every triangle, whichever
 * BVH builder made the tree; triangles are two-sided, the previous triangle
 * is skipped, each new origin is x + eps * (facing normal).  Any origin is
 * accepted; directions are expected near unit length.  Errors: INVALID_ARG,
 * OOM, HIP.  stats (host, nullable) implies a synchronisation. */
int sbr_trace(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_rays *rays, int64_t n_rays, int max_bounces,
              const sbr_trace_opts *opts, sbr_hits *out, sbr_stats *stats);

/* sbr_trace_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same transport, arguments and results as sbr_trace, bit
 * for bit, but the call allocates nothing: its only scratch (the counter
 * block of one streaming launch, 40 KiB) is a static array of the library,
 * one copy per device, looked up when sbr_create sets up the device; the
 * counters are cleared by a fill kernel (no memset node).  Limits: the
 * streaming schedule only (SBR_OPT_WAVEFRONT -> SBR_ERR_UNSUPPORTED: its
 * queues need memory) and trees no deeper than the on-chip traversal stack
 * (28 levels; deeper -> SBR_ERR_UNSUPPORTED, use sbr_trace).  Every call on
 * a device shares that device's scratch, which keeps the last call's
 * contents: calls that overlap on one device (two streams, two threads)
 * race and must be serialised by the caller.  stats (nullable) synchronises
 * the stream and copies the counters to the host; its GPU times stay 0 (no
 * events are created).  Errors as sbr_trace, plus UNSUPPORTED. */
int sbr_trace_noalloc(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_rays *rays, int64_t n_rays, int max_bounces,
                      const sbr_trace_opts *opts, sbr_hits *out, sbr_stats *stats);

/* ------------------------------------------------------------------------ */
/* sbr_po_integrate -- ray-tube physical-optics sum (Eq. po_sum; em5-em6)    */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t struct_size;
    int32_t mode;        /* SBR_MODE_VECTOR or SBR_MODE_PAPER */
    double k_hat[3];     /* incident direction */
    double theta_hat[3]; /* V receive/transmit vector */
    double phi_hat[3];   /* H receive/transmit vector */
    double dA;           /* ray-tube area ds^2 (m^2) */
} sbr_po_desc;

/* Sums over the rays of `hits` (device, as written by sbr_trace; needs
 * n_bounce, tri_first, tri_last, flags, D, d_last, eH_last, eV_last) whose
 * flags have SBR_REC_VALID.  freqs_hz: host [n_freq] (1..4096).  A_out:
 * device [n_freq][2 receive][2 transmit] complex128, i.e. n_freq*8 doubles.
 * The sum is exact-order independent (fixed-point accumulation), so the
 * result is bitwise reproducible.  Errors: INVALID_ARG, OOM, HIP. */
int sbr_po_integrate(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_hits *hits, int64_t n_rays,
                     const sbr_po_desc *desc, const double *freqs_hz, int n_freq, double *A_out);

/* ------------------------------------------------------------------------ */
/* sbr_rcs_sweep -- monostatic RCS over many incidence angles                */
/* ------------------------------------------------------------------------ */

/* Launch parameters of the trace kernels (all have defaults; see
 * sbr_default_tune).  They change speed only, never results. */
typedef struct {
    uint32_t struct_size;
    int32_t schedule;      /* 0 = streaming launch, 1 = one launch per bounce (SBR_OPT_WAVEFRONT) */
    int32_t tile_w;        /* aperture tile of one 64-lane wave: tile_w x (64 / tile_w) rays; 4, 8, 16, 32, 64 */
    int32_t claim_tiles;   /* tiles a wave claims per atomic, 1..64; 0 = automatic: 1 when the tree
                              (nodes and triangles) exceeds 4 MiB, one XCD's L2, else 2 */
    int32_t refill_min;    /* idle lanes that trigger a refill (streaming launch), 1..64 */
    int32_t blocks_per_cu; /* persistent blocks of 256 threads per compute unit; 0 = occupancy limit */
    int32_t chunk_log2;    /* rays per trace/PO chunk = 2^chunk_log2, 16..30; 0 = automatic: a sweep
                              or batch takes 30 when the chunk's record slots (65 bytes a ray, 69 GB)
                              fit in a quarter of the device memory free or already held by the context's
                              or batch's record buffers, else 29.  Records of a chunk stay in
                              device memory between its trace and its PO stage. */
    int32_t reserved;
} sbr_tune;

/* Fills *out with the built-in defaults. */
int sbr_default_tune(sbr_tune *out);


typedef struct {
    uint32_t struct_size;
    const double *theta_deg; /* host [n_angles] */
    const double *phi_deg;   /* host [n_angles] */
    int64_t n_angles;        /* 1 .. 2^24 */
    const double *freqs_hz;  /* host [n_freq] */
    int32_t n_freq;          /* 1 .. 4096 */
    int32_t max_bounces;     /* 1 .. SBR_MAX_BOUNCES */
    double ds;               /* ray spacing (m); 0 = c / (f_max * samples_per_lambda) */
    double samples_per_lambda;
    double eta;              /* aperture margin of Eq. L2 (0.1 if negative) */
    int32_t mode;            /* SBR_MODE_* */
    uint32_t flags;          /* SBR_OPT_* */
    const sbr_tune *tune;    /* NULL = defaults (SBR_OPT_WAVEFRONT still selects that schedule) */
} sbr_sweep;

/* Picks launch parameters for this BVH and sweep by timing candidates on a
 * sample of its angles (at most 16, evenly spaced) with a coordinate search
 * over refill_min, tile_w, claim_tiles and blocks_per_cu.  Results are cached
 * per (device, triangle-count bucket, rays-per-angle bucket, max_bounces) in
 * the context and, if the environment variable SBR_TUNE_CACHE names a file,
 * in that JSON file.  sweep->tune is ignored.  Synchronises the stream.
 * Errors: as sbr_rcs_sweep. */
int sbr_autotune(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_sweep *sweep, sbr_tune *out);

/* For every angle: ray grid of Eqs. L1-L3 over the mesh bounding box (cell
 * centred, one trace at the spacing of the highest frequency), transport,
 * PO sum for every frequency.  A_out: device
 * [n_angles][n_freq][2][2] complex128; sigma_dbsm: device
 * [n_angles][n_freq][2][2] float64 (10 log10 of 4 pi |A|^2, -400 for 0),
 * nullable.  Errors: SAMPLING (ds > lambda_min / 5 without
 * SBR_OPT_ALLOW_UNDERSAMPLING), INVALID_ARG, OOM, HIP.  stats (host,
 * nullable) implies a synchronisation. */
int sbr_rcs_sweep(sbr_ctx *ctx, const sbr_bvh *bvh, const sbr_sweep *sweep, double *A_out, double *sigma_dbsm,
                  sbr_stats *stats);

/* ------------------------------------------------------------------------ */
/* Batched sweeps: many scenes, angles and frequencies in one launch         */
/* ------------------------------------------------------------------------ */

/* Copies the BVHs bvhs[0..n_bvhs) (built with this context, 1 <= n_bvhs <=
 * 65536, at most 2^28 triangles in total) into one multi-scene set *out;
 * scene s of the set is bvhs[s].  Triangle ids of scene s become
 * (sum of n_tris of the earlier scenes) + id.  The inputs stay valid and
 * may be freed afterwards.  A set serves sbr_batch_create only (sbr_trace,
 * sbr_po_integrate and sbr_rcs_sweep reject it); free it with
 * sbr_free_bvh.  Synchronises the stream.  Errors: INVALID_ARG, OVERFLOW,
 * OOM, HIP. */
int sbr_pack_scenes(sbr_ctx *ctx, const sbr_bvh *const *bvhs, int n_bvhs, sbr_bvh **out);

typedef struct {
    int32_t scene;       /* scene index in the set (0 for a single BVH) */
    int32_t n_freq;      /* 1 .. 4096 */
    int64_t freq_offset; /* its frequencies are freqs_hz[freq_offset, freq_offset + n_freq) */
    double theta_deg, phi_deg;
    double ds;           /* ray spacing (m); <= 0: c / (f_max of the item * samples_per_lambda) */
} sbr_batch_item;

typedef struct {
    uint32_t struct_size;
    const sbr_batch_item *items; /* host [n_items] */
    int64_t n_items;             /* 1 .. 2^24 */
    const double *freqs_hz;      /* host [n_freqs_total] */
    int64_t n_freqs_total;
    int32_t max_bounces;         /* 1 .. SBR_MAX_BOUNCES */
    int32_t mode;                /* SBR_MODE_* */
    uint32_t flags;              /* SBR_OPT_* */
    int32_t reserved;
    double samples_per_lambda;   /* used by items with ds <= 0 */
    double eta;                  /* aperture margin of Eq. L2 (0.1 if negative) */
    const sbr_tune *tune;        /* NULL = defaults */
} sbr_batch_desc;

typedef struct sbr_batch sbr_batch; /* planned batch: device buffers + captured graph */

typedef struct {
    int64_t n_items;
    int64_t n_rows;         /* output rows = sum of n_freq over the items */
    int64_t rays;           /* rays over all items */
    int64_t min_item_rays, max_item_rays;
    int32_t n_chunks;       /* trace + PO chunks of the graph */
    int32_t graph_ready;    /* 1 once a graph has been captured for the current outputs and tune */
    int64_t device_bytes;   /* device memory held by the batch */
    sbr_tune tune;          /* launch parameters in use */
} sbr_batch_info;

/* Plans every item of desc against the scene set (or single BVH) `scenes`:
 * per item, the ray grid of Eqs. L1-L3 over its scene's bounding box at its
 * spacing, checked against lambda/5 at its highest frequency (SAMPLING
 * unless SBR_OPT_ALLOW_UNDERSAMPLING).  Items are grouped, in order, into
 * chunks of at most 2^chunk_log2 rays (an item larger than that is a chunk
 * of its own); all device buffers are allocated here.  `scenes` must outlive
 * the batch.  Errors: INVALID_ARG, SAMPLING, OVERFLOW, OOM, HIP. */
int sbr_batch_create(sbr_ctx *ctx, const sbr_bvh *scenes, const sbr_batch_desc *desc, sbr_batch **out);

int sbr_batch_get_info(const sbr_batch *batch, sbr_batch_info *out);

/* Replaces the launch parameters (re-plans tiles and chunks; the next run
 * captures a new graph).  Errors: INVALID_ARG, OOM, HIP. */
int sbr_batch_set_tune(sbr_batch *batch, const sbr_tune *tune);

/* Times candidate launch parameters on a sample of the batch's items (every
 * k-th item, about 1/8 of its rays, at least one item) with a coordinate
 * search over refill_min, tile_w, claim_tiles, blocks_per_cu and chunk_log2,
 * then applies the best with sbr_batch_set_tune and returns it.
 * Synchronises the stream.  Errors: as sbr_batch_run. */
int sbr_batch_autotune(sbr_batch *batch, sbr_tune *out);

/* Runs every item: for each chunk, clear the work counters, one trace
 * launch for all bounces of all its items, the PO launch and the finalize
 * launch.  The whole sequence is captured once into a HIP graph (on a
 * private stream) and replayed on the context stream; a different A_out or
 * sigma_dbsm, or a new tune, triggers a new capture.  A_out: device
 * [n_rows][2][2] complex128, row = (sum of n_freq of the earlier items) + f;
 * sigma_dbsm: device [n_rows][2][2] float64, nullable.  Results are bitwise
 * identical to sbr_rcs_sweep of each item's scene alone and across replays.
 * stats (host, nullable) implies a synchronisation; with a graph only
 * ms_total (GPU time of the graph) is timed, SBR_OPT_NO_GRAPH also fills
 * ms_trace and ms_po.  Concurrent runs of one batch are not allowed.
 * Errors: INVALID_ARG, HIP. */
int sbr_batch_run(sbr_batch *batch, double *A_out, double *sigma_dbsm, sbr_stats *stats);

/* Frees the batch after the device has finished all its work (it does not
 * use the context, which may already be gone).  NULL is accepted.  The
 * context must outlive every other call on the batch. */
void sbr_batch_destroy(sbr_batch *batch);

/* ------------------------------------------------------------------------ */
/* Learned surrogate: Fourier-feature MLP over (theta, phi, f)               */
/* ------------------------------------------------------------------------ */
/* The network maps one point (theta_deg, phi_deg, f_hz) to the co-polarised
 * field (A_HH, A_VV) of the same convention as sbr_rcs_sweep:
 *   xn = 2 (x - lo) / (hi - lo) - 1 per coordinate,
 *   gamma = [sin(2 pi B xn), cos(2 pi B xn)]  (B: [n_ff][3] fixed, N(0, ff_sigma^2)),
 *   h_0 = bf16(gamma), h_l = bf16(act(h_{l-1} bf16(W_l)^T + b_l)), l = 1..depth,
 *   y = h_depth bf16(W_out)^T + b_out (4 outputs),
 *   A_HH = out_scale (y0 + j y1), A_VV = out_scale (y2 + j y3).
 * Products run on the matrix cores in bf16 with fp32 accumulation; master
 * weights are fp32 and trained with Adam (b1 0.9, b2 0.999, eps 1e-8) on the
 * mean squared error of y against targets / out_scale. */

#define SBR_ACT_SILU 0
#define SBR_ACT_RELU 1

typedef struct sbr_mlp sbr_mlp;

typedef struct {
    uint32_t struct_size;
    int32_t n_ff;       /* Fourier features, multiple of 64 in [64, 512] (64) */
    int32_t width;      /* hidden width, multiple of 128 in [128, 1024] (256) */
    int32_t depth;      /* hidden layers, 1..8 (4) */
    int32_t act;        /* SBR_ACT_* */
    int32_t reserved;
    double ff_sigma;    /* standard deviation of the feature matrix B */
    uint64_t seed;      /* seeds B and the initial weights */
    double lo[3], hi[3]; /* input ranges of theta_deg, phi_deg, f_hz */
    double out_scale;   /* output scale (e.g. the RMS of the training targets) */
} sbr_mlp_desc;

typedef struct {
    int64_t n_params;   /* W_1, b_1, ..., W_out, b_out, row-major, fp32 */
    int32_t n_ff, width, depth, act;
    double out_scale;
    int64_t adam_steps;
    double flops_per_point; /* 2 (2 n_ff width + (depth - 1) width^2 + 4 width) */
} sbr_mlp_info;

typedef struct {
    uint32_t struct_size;
    int32_t epochs;
    int32_t batch;      /* points per step, 1..65536 */
    int32_t reserved;
    double lr, lr_min;  /* cosine decay from lr to lr_min over all steps */
    uint64_t seed;      /* shuffling */
} sbr_train_opts;

/* Creates a network with seeded initial weights.  Errors: INVALID_ARG, OOM,
 * HIP. */
int sbr_mlp_create(sbr_ctx *ctx, const sbr_mlp_desc *desc, sbr_mlp **out);
int sbr_mlp_get_info(const sbr_mlp *mlp, sbr_mlp_info *out);
/* Parameters as fp32 host arrays of n_params values (set resets Adam). */
int sbr_mlp_get_params(const sbr_mlp *mlp, float *host, int64_t n);
int sbr_mlp_set_params(sbr_mlp *mlp, const float *host, int64_t n);
/* The feature matrix B, host [n_ff][3]. */
int sbr_mlp_get_features(const sbr_mlp *mlp, float *host);
int sbr_mlp_set_scale(sbr_mlp *mlp, double out_scale);
/* pts: device [n][3] (theta_deg, phi_deg, f_hz); A_out: device [n][2]
 * complex128 (HH, VV).  Errors: INVALID_ARG, OOM, HIP. */
int sbr_mlp_predict(sbr_mlp *mlp, const double *pts, int64_t n, double *A_out);
/* Gradients of the loss over n (1..65536) points: targets device [n][2]
 * complex128; grads device [n_params] fp32; loss (host, nullable) = mean
 * squared error.  Synchronises. */
int sbr_mlp_gradients(sbr_mlp *mlp, const double *pts, const double *targets, int64_t n, float *grads, float *loss);
/* Adam training over shuffled batches; loss_per_epoch host [epochs],
 * nullable.  Synchronises at the end (and once per group of epochs whose
 * shuffled orders exceed 2^24 indices). */
int sbr_mlp_train(sbr_mlp *mlp, const double *pts, const double *targets, int64_t n, const sbr_train_opts *opts,
                  float *loss_per_epoch);
void sbr_mlp_destroy(sbr_mlp *mlp);

/* Dense grid fill: surrogate everywhere, SBR probes judge it per tile, SBR
 * replaces it on every failing tile.  The grid is n_angles directions
 * (theta_deg[a], phi_deg[a]) x n_freq frequencies, cut into tiles of
 * tile_angles consecutive directions x tile_freqs consecutive frequencies.
 * Each angle tile has one probe direction (probe_dir[2 t]: theta, phi) and
 * each frequency tile probes_per_tile probe frequencies (probe_freq
 * [tf * probes_per_tile + q]); SBR at those points (one batch, all of a
 * probe direction's frequencies from one trace) is compared with the
 * network; a tile falls back when, on its probes whose SBR co-polar sigma is
 * at least (largest probe sigma - floor_db), |sigma_net - sigma_sbr| exceeds
 * tol_db in either co-polar channel.  Fallback runs SBR for every point of
 * the failing tiles: per direction, runs of failing tiles separated by
 * passing tiles share one trace when the PO of the passing tiles between
 * them costs less than a trace (the cost ratio is measured on the probe
 * sweep); the points of passing tiles keep the network's value.  Every SBR
 * call traces at spacing ds. */
typedef struct {
    uint32_t struct_size;
    int32_t mode;               /* SBR_MODE_* of every SBR call */
    const double *theta_deg;    /* host [n_angles] */
    const double *phi_deg;      /* host [n_angles] */
    int64_t n_angles;
    const double *freqs_hz;     /* host [n_freq] */
    int32_t n_freq;
    int32_t tile_angles;        /* >= 1 */
    int32_t tile_freqs;         /* >= 1 */
    int32_t probes_per_tile;    /* >= 1 */
    const double *probe_dir;    /* host [n_angle_tiles][2] */
    const double *probe_freq;   /* host [n_freq_tiles * probes_per_tile] */
    int32_t max_bounces;
    uint32_t flags;             /* SBR_OPT_* of every SBR call */
    double ds;                  /* ray spacing (m) */
    double eta;
    double tol_db;              /* 0.5 */
    double floor_db;            /* 40 */
} sbr_fill_desc;

typedef struct {
    int64_t tiles, fallback_tiles, points, fallback_points, probe_points;  /* fallback_points: of failing tiles */
    double ms_predict, ms_probe, ms_check, ms_fallback, ms_total;
    int64_t sbr_rays;           /* rays traced by the probe and fallback SBR calls */
} sbr_fill_stats;

/* A_out: device [n_angles][n_freq][2] complex128 (HH, VV).  tile_err (host
 * [n_angle_tiles][n_freq_tiles], nullable): the largest probe error of each
 * tile (dB); fallback (host, same shape, nullable): 1 where SBR was used.
 * Synchronises.  Errors: as sbr_batch_create and sbr_mlp_predict. */
int sbr_surrogate_fill(sbr_ctx *ctx, const sbr_bvh *bvh, sbr_mlp *mlp, const sbr_fill_desc *desc, double *A_out,
                       double *tile_err, uint8_t *fallback, sbr_fill_stats *stats);

/* ------------------------------------------------------------------------ */
/* Host-only helper (no GPU): the ray grid of one angle, Eqs. L1-L3          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double k_hat[3], theta_hat[3], phi_hat[3];
    double uc, vc, s0, ds;
    int64_t nu, nv; /* rays along phi_hat and theta_hat; ray index = j * nu + i */
} sbr_angle_plan;

/* bbox: lo xyz, hi xyz.  Errors: INVALID_ARG (ds <= 0, non-finite input). */
int sbr_plan_angle(const double bbox[6], double theta_deg, double phi_deg, double ds, double eta,
                   sbr_angle_plan *out);

#ifdef __cplusplus
}
#endif

#endif /* SBR_H */
