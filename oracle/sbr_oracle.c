/*
 * CPU oracle for the SBR trace-integrate path (arXiv 2604.09243).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header or constant table with the HIP library.
 *
 * What it computes, and where the paper defines it:
 *   - mesh preparation: edge vectors, unit normals, bounding box, offset
 *     epsilon (Sec. 4 BVH paragraph: leaves reference contiguous triangle
 *     ranges; Sec. 4 offset "epsilon along the normal");
 *   - incidence frame and aperture ray grid, Eqs. (L1)-(L3) (Sec. 4);
 *   - multi-bounce specular transport, Algorithm 2 (Sec. 4), with the
 *     closest hit found by testing EVERY triangle (brute force) or, in the
 *     fast mode, through the binned-SAH / median BVH of Algorithm 1 and the
 *     SAH cost equation (Sec. 4);
 *   - the ray-tube physical-optics sum: Eq. (po_sum) literally (PAPER mode),
 *     or Eqs. (em5)-(em6) applied to each ray tube's footprint on its last
 *     facet with the polarisation carried through every PEC reflection
 *     (VECTOR mode; polarimetric scattering is listed as future work in
 *     Sec. 7, so this mode is a reading, stated in the design notes);
 *   - sigma = 4 pi |A|^2 (Sec. 4, trace-integrate paragraph).
 *
 * Precision: the intersection test and the ray geometry (origin, direction)
 * are float32 with a fixed operation order and no contraction (compile with
 * -ffp-contract=off), because that arithmetic decides integers (which
 * triangle is hit, how many bounces) and the HIP path must take the same
 * decisions.  Path length, polarisation and the PO sum are float64.
 *
 * Hit rule (a reading: the paper fixes no rounding).  A triangle is hit when
 * the float32 Moller-Trumbore test accepts it AND the float32 hit point
 * x = o + t d lies inside the triangle's axis-aligned box widened by
 * P = fl32(2^-20 M) on every side, M = X + C + 1.5 |diag| (X = largest
 * |coordinate| of the scene's box, C = that of its centre): every ray
 * origin and hit point of a sweep lies within M.  The widening is about 16
 * float32 units of that scale, many times the rounding of a well
 * conditioned test; only hits whose float32 point has drifted off the
 * triangle (grazing rays, slivers seen from afar) are refused, and the
 * closest hit is then a minimum that a bounding-volume tree can find
 * exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_C0 299792458.0
#define ORC_PI 3.14159265358979323846

/* record flag bits */
#define ORC_F_VALID 1
#define ORC_F_TRAPPED 2
#define ORC_F_BACK_LAST 4 /* facing normal at the last hit is -n */
#define ORC_F_EDGE 8      /* edge-ambiguous at some query (diagnostic) */

/* trace option bits */
#define ORC_USE_BVH 1
#define ORC_DROP_TRAPPED 2
#define ORC_PAPER_PATH 4
#define ORC_EDGE_DIAG 8
/* Precision study of Sec. 6 (not the method's arithmetic): accumulate the
 * path P and form D in float32 (orc_trace), and form the phase k D in float32
 * (orc_po, or-ed into mode). */
#define ORC_FP32_PATH 16
/* Brute force with the Moller-Trumbore conditions only (no box rule), to
 * show which hits the rule refuses; not the method. */
#define ORC_MT_ONLY 32

typedef struct {
    float lo[3], hi[3];
    int32_t left, right; /* left < 0: leaf */
    int32_t first, count;
} orc_node;

typedef struct {
    int64_t nt;
    float *v0, *e1, *e2, *n; /* [nt*3] */
    unsigned char *degen;    /* [nt] */
    double bbox[6];
    double diag;
    float eps;
    float pbox;  /* the hit rule's widening P */
    double xmax; /* largest |coordinate| of any widened triangle box */
    int64_t n_degen;
    /* optional BVH (fast mode) */
    orc_node *nodes;
    int64_t n_nodes;
    int32_t *order; /* leaf order -> triangle id */
    int depth;
} orc_mesh;

/* ------------------------------------------------------------------------ */
/* Mesh preparation                                                          */
/* ------------------------------------------------------------------------ */

/* Returns NULL on invalid input (non-finite vertex or index out of range);
 * *status = 0 ok, -2 invalid mesh, -4 out of memory. */
orc_mesh *orc_mesh_new(const float *V, int64_t nv, const int32_t *T, int64_t nt, int *status)
{
    *status = 0;
    for (int64_t i = 0; i < nv * 3; i++)
        if (!isfinite(V[i])) { *status = -2; return NULL; }
    for (int64_t i = 0; i < nt * 3; i++)
        if (T[i] < 0 || T[i] >= nv) { *status = -2; return NULL; }
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    if (!m) { *status = -4; return NULL; }
    m->nt = nt;
    m->v0 = (float *)malloc(sizeof(float) * 3 * (nt ? nt : 1));
    m->e1 = (float *)malloc(sizeof(float) * 3 * (nt ? nt : 1));
    m->e2 = (float *)malloc(sizeof(float) * 3 * (nt ? nt : 1));
    m->n = (float *)malloc(sizeof(float) * 3 * (nt ? nt : 1));
    m->degen = (unsigned char *)malloc(nt ? nt : 1);
    if (!m->v0 || !m->e1 || !m->e2 || !m->n || !m->degen) { *status = -4; return NULL; }

    /* bounding box over every vertex referenced by a triangle */
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = 0; j < nt; j++)
        for (int c = 0; c < 3; c++) {
            const float *p = V + 3 * (int64_t)T[3 * j + c];
            for (int a = 0; a < 3; a++) {
                if (p[a] < lo[a]) lo[a] = p[a];
                if (p[a] > hi[a]) hi[a] = p[a];
            }
        }
    if (nt == 0) { lo[0] = lo[1] = lo[2] = hi[0] = hi[1] = hi[2] = 0.0; }
    for (int a = 0; a < 3; a++) { m->bbox[a] = lo[a]; m->bbox[3 + a] = hi[a]; }
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    m->diag = sqrt((dx * dx + dy * dy) + dz * dz);
    /* offset distance: 1e-5 of the scene diagonal (the paper leaves its value open) */
    m->eps = (float)(1e-5 * m->diag);
    /* hit rule widening P = fl32(2^-20 M), M = (X + C) + 1.5 |diag| */
    {
        double X = 0.0, C = 0.0;
        for (int a = 0; a < 3; a++) {
            X = fmax(X, fmax(fabs(lo[a]), fabs(hi[a])));
            C = fmax(C, fabs(0.5 * (lo[a] + hi[a])));
        }
        double M = (X + C) + 1.5 * m->diag;
        m->pbox = (float)(M * 0x1p-20);
        m->xmax = X + 2.0 * (double)m->pbox;
    }
    double amin = 1e-12 * m->diag * m->diag;

    for (int64_t j = 0; j < nt; j++) {
        const float *a = V + 3 * (int64_t)T[3 * j + 0];
        const float *b = V + 3 * (int64_t)T[3 * j + 1];
        const float *c = V + 3 * (int64_t)T[3 * j + 2];
        float *v0 = m->v0 + 3 * j, *e1 = m->e1 + 3 * j, *e2 = m->e2 + 3 * j, *n = m->n + 3 * j;
        for (int k = 0; k < 3; k++) {
            v0[k] = a[k];
            e1[k] = b[k] - a[k];
            e2[k] = c[k] - a[k];
        }
        /* normal of the float32 edges, evaluated in float64 */
        double cx = (double)e1[1] * (double)e2[2] - (double)e1[2] * (double)e2[1];
        double cy = (double)e1[2] * (double)e2[0] - (double)e1[0] * (double)e2[2];
        double cz = (double)e1[0] * (double)e2[1] - (double)e1[1] * (double)e2[0];
        double len = sqrt((cx * cx + cy * cy) + cz * cz);
        int dg = !(0.5 * len >= amin) || !(len > 0.0);
        m->degen[j] = (unsigned char)dg;
        if (dg) {
            m->n_degen++;
            n[0] = n[1] = n[2] = 0.0f;
        } else {
            n[0] = (float)(cx / len);
            n[1] = (float)(cy / len);
            n[2] = (float)(cz / len);
        }
    }
    return m;
}

static void free_bvh(orc_mesh *m)
{
    free(m->nodes);
    free(m->order);
    m->nodes = NULL;
    m->order = NULL;
    m->n_nodes = 0;
}

void orc_mesh_free(orc_mesh *m)
{
    if (!m) return;
    free(m->v0); free(m->e1); free(m->e2); free(m->n); free(m->degen);
    free_bvh(m);
    free(m);
}

void orc_mesh_info(const orc_mesh *m, double bbox[6], float *eps, int64_t *n_degen, int64_t *n_nodes, int *depth)
{
    memcpy(bbox, m->bbox, sizeof(double) * 6);
    *eps = m->eps;
    *n_degen = m->n_degen;
    *n_nodes = m->n_nodes;
    *depth = m->depth;
}

void orc_mesh_normals(const orc_mesh *m, float *out)
{
    memcpy(out, m->n, sizeof(float) * 3 * m->nt);
}

/* Boxes (lo.xyz, hi.xyz) of the leaves of the mesh's BVH, in node order, into
 * out[6 * cap]; returns the number of leaves (0 without a BVH).  Used only to
 * price traversal work, never in the method itself. */
int64_t orc_mesh_leaf_boxes(const orc_mesh *m, double *out, int64_t cap)
{
    int64_t k = 0;
    for (int64_t i = 0; i < m->n_nodes; ++i) {
        const orc_node *nd = &m->nodes[i];
        if (nd->left >= 0) continue;
        if (k < cap)
            for (int a = 0; a < 3; ++a) {
                out[6 * k + a] = nd->lo[a];
                out[6 * k + 3 + a] = nd->hi[a];
            }
        ++k;
    }
    return k;
}

/* ------------------------------------------------------------------------ */
/* BVH of Algorithm 1 (fast mode): median split or binned SAH                 */
/* ------------------------------------------------------------------------ */

/* The hit rule's box of triangle j: the box of its float32 corners v0,
 * v0 + e1, v0 + e2 (each sum rounded to float32), widened by P, in float32. */
static void rule_box(const orc_mesh *m, int64_t j, float lo[3], float hi[3])
{
    const float *v0 = m->v0 + 3 * j, *e1 = m->e1 + 3 * j, *e2 = m->e2 + 3 * j;
    for (int a = 0; a < 3; a++) {
        float p1 = v0[a] + e1[a], p2 = v0[a] + e2[a];
        float mn = v0[a], mx = v0[a];
        if (p1 < mn) mn = p1;
        if (p2 < mn) mn = p2;
        if (p1 > mx) mx = p1;
        if (p2 > mx) mx = p2;
        lo[a] = mn - m->pbox;
        hi[a] = mx + m->pbox;
    }
}

typedef struct {
    const orc_mesh *m;
    float *tlo, *thi; /* per-triangle boxes of the hit rule */
    float *cen;       /* centroids */
    int32_t *idx;     /* working permutation */
    orc_node *nodes;
    int64_t n_nodes, cap;
    int nleaf, nbins, rule, maxdepth;
} bvh_build;

static double box_area(const float lo[3], const float hi[3])
{
    double x = (double)hi[0] - lo[0], y = (double)hi[1] - lo[1], z = (double)hi[2] - lo[2];
    if (x < 0 || y < 0 || z < 0) return 0.0;
    return 2.0 * (x * y + y * z + z * x);
}

static int cmp_axis;
static const float *cmp_cen;
static int cmp_centroid(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    float ca = cmp_cen[3 * i + cmp_axis], cb = cmp_cen[3 * j + cmp_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return (i > j) - (i < j);
}

/* Builds the subtree over idx[first, first+count) and returns its node id.
 * Nodes are appended depth-first, left subtree first, so the array is in
 * preorder with the left child right after its parent. */
static int32_t build_rec(bvh_build *B, int32_t first, int32_t count, int depth)
{
    if (B->n_nodes == B->cap) {
        B->cap *= 2;
        B->nodes = (orc_node *)realloc(B->nodes, sizeof(orc_node) * B->cap);
    }
    int32_t id = (int32_t)B->n_nodes++;
    orc_node nd;
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int a = 0; a < 3; a++) { nd.lo[a] = INFINITY; nd.hi[a] = -INFINITY; }
    for (int32_t k = first; k < first + count; k++) {
        int32_t t = B->idx[k];
        for (int a = 0; a < 3; a++) {
            if (B->tlo[3 * t + a] < nd.lo[a]) nd.lo[a] = B->tlo[3 * t + a];
            if (B->thi[3 * t + a] > nd.hi[a]) nd.hi[a] = B->thi[3 * t + a];
            if (B->cen[3 * t + a] < clo[a]) clo[a] = B->cen[3 * t + a];
            if (B->cen[3 * t + a] > chi[a]) chi[a] = B->cen[3 * t + a];
        }
    }
    if (depth > B->maxdepth) B->maxdepth = depth;
    if (count <= B->nleaf) {
        nd.left = nd.right = -1;
        nd.first = first;
        nd.count = count;
        B->nodes[id] = nd;
        return id;
    }
    int32_t mid = -1;
    if (B->rule == 1) {
        /* binned SAH: C = C_T + SA(L)/SA(P) N_L C_I + SA(R)/SA(P) N_R C_I */
        const double CT = 1.0, CI = 1.0;
        double sap = box_area(nd.lo, nd.hi);
        double best = INFINITY;
        int bax = -1, bsplit = -1;
        int NB = B->nbins;
        for (int a = 0; a < 3; a++) {
            double ext = (double)chi[a] - clo[a];
            if (!(ext > 0.0)) continue;
            int cnt[64];
            float blo[64][3], bhi[64][3];
            for (int b = 0; b < NB; b++) {
                cnt[b] = 0;
                for (int c = 0; c < 3; c++) { blo[b][c] = INFINITY; bhi[b][c] = -INFINITY; }
            }
            for (int32_t k = first; k < first + count; k++) {
                int32_t t = B->idx[k];
                int b = (int)(NB * (((double)B->cen[3 * t + a] - clo[a]) / ext));
                if (b >= NB) b = NB - 1;
                if (b < 0) b = 0;
                cnt[b]++;
                for (int c = 0; c < 3; c++) {
                    if (B->tlo[3 * t + c] < blo[b][c]) blo[b][c] = B->tlo[3 * t + c];
                    if (B->thi[3 * t + c] > bhi[b][c]) bhi[b][c] = B->thi[3 * t + c];
                }
            }
            for (int s = 1; s < NB; s++) {
                float llo[3] = {INFINITY, INFINITY, INFINITY}, lhi[3] = {-INFINITY, -INFINITY, -INFINITY};
                float rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
                int nl = 0, nr = 0;
                for (int b = 0; b < NB; b++) {
                    float *xlo = b < s ? llo : rlo, *xhi = b < s ? lhi : rhi;
                    if (b < s) nl += cnt[b]; else nr += cnt[b];
                    for (int c = 0; c < 3; c++) {
                        if (blo[b][c] < xlo[c]) xlo[c] = blo[b][c];
                        if (bhi[b][c] > xhi[c]) xhi[c] = bhi[b][c];
                    }
                }
                if (nl == 0 || nr == 0) continue;
                double cost = CT + box_area(llo, lhi) / sap * nl * CI + box_area(rlo, rhi) / sap * nr * CI;
                if (cost < best) { best = cost; bax = a; bsplit = s; }
            }
        }
        if (bax >= 0) {
            double ext = (double)chi[bax] - clo[bax];
            int32_t i = first, j = first + count - 1;
            while (i <= j) {
                int32_t t = B->idx[i];
                int b = (int)(NB * (((double)B->cen[3 * t + bax] - clo[bax]) / ext));
                if (b >= NB) b = NB - 1;
                if (b < 0) b = 0;
                if (b < bsplit) i++;
                else { int32_t tmp = B->idx[i]; B->idx[i] = B->idx[j]; B->idx[j] = tmp; j--; }
            }
            mid = i;
            if (mid == first || mid == first + count) mid = -1;
        }
    }
    if (mid < 0) {
        /* median split of the centroids along the longest centroid-box axis */
        int ax = 0;
        double e0 = (double)chi[0] - clo[0], e1 = (double)chi[1] - clo[1], e2 = (double)chi[2] - clo[2];
        if (e1 > e0 && e1 >= e2) ax = 1;
        else if (e2 > e0 && e2 > e1) ax = 2;
        cmp_axis = ax;
        cmp_cen = B->cen;
        qsort(B->idx + first, (size_t)count, sizeof(int32_t), cmp_centroid);
        mid = first + count / 2;
    }
    B->nodes[id] = nd; /* placeholder; children filled below */
    int32_t l = build_rec(B, first, mid - first, depth + 1);
    int32_t r = build_rec(B, mid, first + count - mid, depth + 1);
    B->nodes[id].left = l;
    B->nodes[id].right = r;
    B->nodes[id].first = first;
    B->nodes[id].count = count;
    return id;
}

/* rule: 0 = median split, 1 = binned SAH.  A triangle's box is exactly the
 * widened box of the hit rule, so every accepted hit point lies inside the
 * box of each node above its triangle. */
int orc_mesh_build_bvh(orc_mesh *m, int rule, int nleaf, int nbins)
{
    free_bvh(m);
    if (nbins > 64) nbins = 64;
    if (nbins < 2) nbins = 2;
    if (nleaf < 1) nleaf = 1;
    bvh_build B;
    memset(&B, 0, sizeof(B));
    B.m = m;
    int64_t nt = m->nt;
    int64_t nlive = 0;
    for (int64_t j = 0; j < nt; j++) nlive += !m->degen[j];
    B.tlo = (float *)malloc(sizeof(float) * 3 * (nt + 1));
    B.thi = (float *)malloc(sizeof(float) * 3 * (nt + 1));
    B.cen = (float *)malloc(sizeof(float) * 3 * (nt + 1));
    B.idx = (int32_t *)malloc(sizeof(int32_t) * (nlive + 1));
    B.cap = 1024;
    B.nodes = (orc_node *)malloc(sizeof(orc_node) * B.cap);
    B.nleaf = nleaf;
    B.nbins = nbins;
    B.rule = rule;
    int64_t w = 0;
    for (int64_t j = 0; j < nt; j++) {
        rule_box(m, j, B.tlo + 3 * j, B.thi + 3 * j);
        const float *v0 = m->v0 + 3 * j, *e1 = m->e1 + 3 * j, *e2 = m->e2 + 3 * j;
        for (int a = 0; a < 3; a++) {
            double p0 = v0[a], p1 = (double)v0[a] + e1[a], p2 = (double)v0[a] + e2[a];
            B.cen[3 * j + a] = (float)((p0 + p1 + p2) / 3.0);
        }
        if (!m->degen[j]) B.idx[w++] = (int32_t)j;
    }
    if (nlive > 0) build_rec(&B, 0, (int32_t)nlive, 0);
    m->nodes = B.nodes;
    m->n_nodes = B.n_nodes;
    m->order = B.idx;
    m->depth = B.maxdepth;
    free(B.tlo); free(B.thi); free(B.cen);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Incidence frame and aperture grid, Eqs. (L1)-(L3)                         */
/* ------------------------------------------------------------------------ */

/* theta: polar angle from +z, phi: azimuth (degrees).  The radar sits along
 * r = (sin t cos p, sin t sin p, cos t); the wave travels along k = -r.
 * The aperture axes are u = phi_hat and v = theta_hat, so (u, v, k) is
 * right-handed; the transmit/receive polarisations are H = phi_hat and
 * V = theta_hat. */
void orc_frame(double theta_deg, double phi_deg, double k[3], double th_hat[3], double ph_hat[3])
{
    double th = theta_deg * (ORC_PI / 180.0);
    double ph = phi_deg * (ORC_PI / 180.0);
    double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    k[0] = -(st * cp);
    k[1] = -(st * sp);
    k[2] = -ct;
    th_hat[0] = ct * cp;
    th_hat[1] = ct * sp;
    th_hat[2] = -st;
    ph_hat[0] = -sp;
    ph_hat[1] = cp;
    ph_hat[2] = 0.0;
}

static double dot3d(const double a[3], const double b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

/* Eq. (L1): project the eight bounding-box corners on u and v; Eq. (L2):
 * widen by (1 + eta); Eq. (L3): N = ceil(L~ / ds).  The grid is cell
 * centred on the middle of the projected box; the launch plane sits 1% of
 * the box diagonal in front of the nearest corner. */
void orc_aperture(const double bbox[6], double theta_deg, double phi_deg, double ds, double eta,
                  int64_t *Nu, int64_t *Nv, double *uc, double *vc, double *s0)
{
    double k[3], v[3], u[3];
    orc_frame(theta_deg, phi_deg, k, v, u);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, kmin = INFINITY;
    for (int c = 0; c < 8; c++) {
        double p[3] = {bbox[(c & 1) ? 3 : 0], bbox[(c & 2) ? 4 : 1], bbox[(c & 4) ? 5 : 2]};
        double pu = dot3d(p, u), pv = dot3d(p, v), pk = dot3d(p, k);
        if (pu < umin) umin = pu;
        if (pu > umax) umax = pu;
        if (pv < vmin) vmin = pv;
        if (pv > vmax) vmax = pv;
        if (pk < kmin) kmin = pk;
    }
    double Lu = umax - umin, Lv = vmax - vmin;
    double Lut = (1.0 + eta) * Lu, Lvt = (1.0 + eta) * Lv;
    *Nu = (int64_t)ceil(Lut / ds);
    *Nv = (int64_t)ceil(Lvt / ds);
    if (*Nu < 1) *Nu = 1;
    if (*Nv < 1) *Nv = 1;
    *uc = 0.5 * (umin + umax);
    *vc = 0.5 * (vmin + vmax);
    double ex = bbox[3] - bbox[0], ey = bbox[4] - bbox[1], ez = bbox[5] - bbox[2];
    double diag = sqrt((ex * ex + ey * ey) + ez * ez);
    *s0 = kmin - 0.01 * diag;
}

/* Ray (i, j) of the grid, ray index j*Nu + i.  Origins are formed in float64
 * and rounded once to float32; every ray of the bundle has d = fl32(k). */
void orc_gen_rays(const double bbox[6], double theta_deg, double phi_deg, double ds, double eta,
                  float *o, float d[3])
{
    double k[3], v[3], u[3];
    orc_frame(theta_deg, phi_deg, k, v, u);
    int64_t Nu, Nv;
    double uc, vc, s0;
    orc_aperture(bbox, theta_deg, phi_deg, ds, eta, &Nu, &Nv, &uc, &vc, &s0);
    for (int64_t j = 0; j < Nv; j++) {
        double vj = vc + (((double)j + 0.5) - 0.5 * (double)Nv) * ds;
        for (int64_t i = 0; i < Nu; i++) {
            double ui = uc + (((double)i + 0.5) - 0.5 * (double)Nu) * ds;
            float *p = o + 3 * (j * Nu + i);
            for (int a = 0; a < 3; a++) p[a] = (float)((ui * u[a] + vj * v[a]) + s0 * k[a]);
        }
    }
    for (int a = 0; a < 3; a++) d[a] = (float)k[a];
}

/* ------------------------------------------------------------------------ */
/* Closest hit                                                               */
/* ------------------------------------------------------------------------ */

/* Moller-Trumbore in float32, fixed evaluation order, no contraction. */
static inline int tri_hit(const orc_mesh *m, int64_t j, const float o[3], const float d[3], float *t_out)
{
    const float *v0 = m->v0 + 3 * j, *e1 = m->e1 + 3 * j, *e2 = m->e2 + 3 * j;
    float px = d[1] * e2[2] - d[2] * e2[1];
    float py = d[2] * e2[0] - d[0] * e2[2];
    float pz = d[0] * e2[1] - d[1] * e2[0];
    float det = (e1[0] * px + e1[1] * py) + e1[2] * pz;
    if (det == 0.0f) return 0;
    float sx = o[0] - v0[0], sy = o[1] - v0[1], sz = o[2] - v0[2];
    float un = (sx * px + sy * py) + sz * pz;
    float qx = sy * e1[2] - sz * e1[1];
    float qy = sz * e1[0] - sx * e1[2];
    float qz = sx * e1[1] - sy * e1[0];
    float vn = (d[0] * qx + d[1] * qy) + d[2] * qz;
    float tn = (e2[0] * qx + e2[1] * qy) + e2[2] * qz;
    float inv = 1.0f / det;
    float u = un * inv, v = vn * inv, t = tn * inv;
    if (u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t > 0.0f && t < INFINITY) {
        *t_out = t;
        return 1;
    }
    return 0;
}

typedef struct {
    int64_t box_tests, tri_tests;
} orc_count;

/* The hit rule's second condition: the float32 hit point o + t d (the point
 * the bounce update uses) inside the triangle's widened box. */
static inline int point_in_rule_box(const orc_mesh *m, int64_t j, const float o[3], const float d[3], float t)
{
    float lo[3], hi[3];
    rule_box(m, j, lo, hi);
    for (int a = 0; a < 3; a++) {
        float x = o[a] + t * d[a];
        if (!(x >= lo[a] && x <= hi[a])) return 0;
    }
    return 1;
}

static inline int rule_hit(const orc_mesh *m, int64_t j, const float o[3], const float d[3], float *t_out)
{
    float t;
    if (!tri_hit(m, j, o, d, &t) || !point_in_rule_box(m, j, o, d, t)) return 0;
    *t_out = t;
    return 1;
}

/* Every triangle, in increasing id order; ties on t keep the smaller id. */
static int32_t closest_brute(const orc_mesh *m, const float o[3], const float d[3], int32_t skip,
                             float *tbest, orc_count *cnt, int mt_only)
{
    float best = INFINITY;
    int32_t bj = -1;
    for (int64_t j = 0; j < m->nt; j++) {
        if (m->degen[j] || j == skip) continue;
        float t;
        cnt->tri_tests++;
        if ((mt_only ? tri_hit(m, j, o, d, &t) : rule_hit(m, j, o, d, &t)) && t < best) {
            best = t;
            bj = (int32_t)j;
        }
    }
    *tbest = best;
    return bj;
}

/* Slab test in float64 against a node box widened by E on every side; the
 * interval is clipped to [0, tmax_in]. */
static int box_hit(const orc_node *nd, const double o[3], const double d[3], double E, double tmax_in,
                   double *tenter)
{
    double tmin = 0.0, tmax = tmax_in;
    for (int a = 0; a < 3; a++) {
        double lo = (double)nd->lo[a] - E, hi = (double)nd->hi[a] + E;
        if (d[a] == 0.0) {
            if (o[a] < lo || o[a] > hi) return 0;
            continue;
        }
        double t0 = (lo - o[a]) / d[a], t1 = (hi - o[a]) / d[a];
        if (t0 > t1) { double x = t0; t0 = t1; t1 = x; }
        if (t0 > tmin) tmin = t0;
        if (t1 < tmax) tmax = t1;
    }
    *tenter = tmin;
    return tmin <= tmax;
}

/* The same minimum as closest_brute, through the tree.  An accepted hit at t
 * has its float32 point x inside every box above its triangle, and the exact
 * point o + t d lies within 2^-24 (2 |x| + |o|) of x on each axis, less than
 * E = 2^-21 (xmax + |o|); the float64 slab test of the box widened by E
 * (rounding near 2^-52 of the same magnitudes) therefore meets the exact
 * point, so a box is skipped only when it holds no accepted hit with t at
 * most the best one so far (ties included: the entry is compared with >). */
static int32_t closest_bvh(const orc_mesh *m, const float o[3], const float d[3], int32_t skip,
                           float *tbest, orc_count *cnt)
{
    float best = INFINITY;
    int32_t bj = -1;
    if (m->n_nodes == 0) { *tbest = best; return -1; }
    double od[3] = {o[0], o[1], o[2]}, dd[3] = {d[0], d[1], d[2]};
    double om = fmax(fabs(od[0]), fmax(fabs(od[1]), fabs(od[2])));
    double E = 0x1p-21 * (m->xmax + om);
    int32_t stack[256];
    int sp = 0;
    double te;
    cnt->box_tests++;
    if (!box_hit(&m->nodes[0], od, dd, E, INFINITY, &te)) { *tbest = best; return -1; }
    stack[sp++] = 0;
    while (sp > 0) {
        int32_t ni = stack[--sp];
        const orc_node *nd = &m->nodes[ni];
        if (nd->left < 0) {
            for (int32_t k = nd->first; k < nd->first + nd->count; k++) {
                int32_t j = m->order[k];
                if (j == skip) continue;
                float t;
                cnt->tri_tests++;
                if (rule_hit(m, j, o, d, &t) && (t < best || (t == best && j < bj))) {
                    best = t;
                    bj = j;
                }
            }
            continue;
        }
        double lim = (double)best;
        double tl, tr;
        cnt->box_tests += 2;
        int hl = box_hit(&m->nodes[nd->left], od, dd, E, lim, &tl);
        int hr = box_hit(&m->nodes[nd->right], od, dd, E, lim, &tr);
        /* push the far child first so the near one is visited next */
        if (hl && hr) {
            if (tl <= tr) { stack[sp++] = nd->right; stack[sp++] = nd->left; }
            else { stack[sp++] = nd->left; stack[sp++] = nd->right; }
        } else if (hl) stack[sp++] = nd->left;
        else if (hr) stack[sp++] = nd->right;
    }
    *tbest = best;
    return bj;
}

/* Diagnostic of how close a query came to an ambiguous decision, in float64:
 * a triangle in front of the ray (up to the closest t) whose barycentric
 * margin min(u, v, 1-u-v) lies within 1e-6 of zero, or a second triangle
 * hit within a relative 1e-6 of the closest t. */
static int edge_ambiguous(const orc_mesh *m, const float o[3], const float d[3], int32_t skip, float tc, int32_t jc)
{
    double lim = (tc < INFINITY) ? (double)tc * (1.0 + 1e-6) : INFINITY;
    for (int64_t j = 0; j < m->nt; j++) {
        if (m->degen[j] || j == skip) continue;
        const float *v0 = m->v0 + 3 * j, *e1 = m->e1 + 3 * j, *e2 = m->e2 + 3 * j;
        double px = (double)d[1] * e2[2] - (double)d[2] * e2[1];
        double py = (double)d[2] * e2[0] - (double)d[0] * e2[2];
        double pz = (double)d[0] * e2[1] - (double)d[1] * e2[0];
        double det = (e1[0] * px + e1[1] * py) + e1[2] * pz;
        if (det == 0.0) continue;
        double sx = (double)o[0] - v0[0], sy = (double)o[1] - v0[1], sz = (double)o[2] - v0[2];
        double qx = sy * e1[2] - sz * e1[1], qy = sz * e1[0] - sx * e1[2], qz = sx * e1[1] - sy * e1[0];
        double u = ((sx * px + sy * py) + sz * pz) / det;
        double v = ((d[0] * qx + d[1] * qy) + d[2] * qz) / det;
        double t = ((e2[0] * qx + e2[1] * qy) + e2[2] * qz) / det;
        if (!(t > 0.0) || t > lim) continue;
        double w = 1.0 - u - v;
        double mn = fmin(u, fmin(v, w));
        if (mn > -1e-6 && mn < 1e-6) return 1;
        if (mn >= 0.0 && j != jc && tc < INFINITY && fabs(t - (double)tc) <= 1e-6 * (double)tc) return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Multi-bounce transport, Algorithm 2                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t *nb;        /* [n] bounce count N */
    int32_t *tri_first; /* [n] */
    int32_t *tri_last;  /* [n] */
    int32_t *flags;     /* [n] ORC_F_* */
    double *path;       /* [n] accumulated one-way path P */
    double *D;          /* [n] round-trip phase path */
    float *d_last;      /* [n*3] direction arriving at the last hit */
    float *x_last;      /* [n*3] last hit point */
    double *eH_last;    /* [n*3] H-transmit polarisation arriving at the last hit */
    double *eV_last;    /* [n*3] V-transmit polarisation arriving at the last hit */
    int32_t *tri_path;  /* [n*bmax] triangle hit at each bounce, -1 after the end */
    int64_t counters[4];/* out: queries, box tests, triangle tests, edge-ambiguous rays */
} orc_trace_out;

static double dotk(const double k[3], const float v[3])
{
    return (k[0] * (double)v[0] + k[1] * (double)v[1]) + k[2] * (double)v[2];
}

int orc_trace(const orc_mesh *m, int64_t n, const float *o_in, const float *d_in,
              const double eH0[3], const double eV0[3], const double k[3], int bmax, int opts,
              orc_trace_out *out)
{
    if (bmax < 1 || bmax > 127) return -1;
    if ((opts & ORC_USE_BVH) && m->n_nodes == 0 && m->nt > 0) return -1;
    int64_t q_tot = 0, box_tot = 0, tri_tot = 0, edge_tot = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : q_tot, box_tot, tri_tot, edge_tot)
    for (int64_t r = 0; r < n; r++) {
        float o[3] = {o_in[3 * r], o_in[3 * r + 1], o_in[3 * r + 2]};
        float d[3] = {d_in[3 * r], d_in[3 * r + 1], d_in[3 * r + 2]};
        double eH[3] = {eH0[0], eH0[1], eH0[2]}, eV[3] = {eV0[0], eV0[1], eV0[2]};
        double P = 0.0;
        int32_t N = 0, first = -1, prev = -1, flags = 0;
        float nfp[3] = {0, 0, 0};
        float dl[3] = {0, 0, 0}, xl[3] = {0, 0, 0};
        double eHl[3] = {0, 0, 0}, eVl[3] = {0, 0, 0};
        orc_count cnt = {0, 0};
        int64_t queries = 0;
        int edge = 0;
        for (int b = 1; b <= bmax; b++) {
            float t;
            queries++;
            int32_t j = (opts & ORC_USE_BVH) ? closest_bvh(m, o, d, prev, &t, &cnt)
                                             : closest_brute(m, o, d, prev, &t, &cnt, (opts & ORC_MT_ONLY) != 0);
            if ((opts & ORC_EDGE_DIAG) && edge_ambiguous(m, o, d, prev, t, j)) edge = 1;
            if (j < 0) break;
            float x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
            const int fp32 = (opts & ORC_FP32_PATH) != 0;
            P = fp32 ? (double)((float)P + t) : P + (double)t;
            if (b >= 2 && !(opts & ORC_PAPER_PATH)) {
                /* first-order correction for starting the segment eps off the surface */
                if (fp32) {
                    float c32 = (nfp[0] * d[0] + nfp[1] * d[1]) + nfp[2] * d[2];
                    P = (double)((float)P + m->eps * c32);
                } else {
                    double c = ((double)nfp[0] * d[0] + (double)nfp[1] * d[1]) + (double)nfp[2] * d[2];
                    P = P + (double)m->eps * c;
                }
            }
            N = N + 1;
            if (N == 1) first = j;
            if (out->tri_path) out->tri_path[r * bmax + (b - 1)] = j;
            for (int a = 0; a < 3; a++) {
                dl[a] = d[a];
                xl[a] = x[a];
                eHl[a] = eH[a];
                eVl[a] = eV[a];
            }
            const float *nn = m->n + 3 * (int64_t)j;
            float dn = (d[0] * nn[0] + d[1] * nn[1]) + d[2] * nn[2];
            float nf[3];
            if (dn < 0.0f) { nf[0] = nn[0]; nf[1] = nn[1]; nf[2] = nn[2]; flags &= ~ORC_F_BACK_LAST; }
            else { nf[0] = -nn[0]; nf[1] = -nn[1]; nf[2] = -nn[2]; flags |= ORC_F_BACK_LAST; }
            /* specular reflection d' = d - 2 (d.n) n */
            float s = 2.0f * dn;
            for (int a = 0; a < 3; a++) d[a] = d[a] - s * nn[a];
            /* PEC reflection of the field: e' = 2 (n.e) n - e (tangential part flips) */
            double nd[3] = {nn[0], nn[1], nn[2]};
            double cH = 2.0 * dot3d(nd, eH), cV = 2.0 * dot3d(nd, eV);
            for (int a = 0; a < 3; a++) {
                eH[a] = cH * nd[a] - eH[a];
                eV[a] = cV * nd[a] - eV[a];
            }
            /* new origin: eps off the surface on the side the ray arrived from */
            for (int a = 0; a < 3; a++) o[a] = x[a] + m->eps * nf[a];
            for (int a = 0; a < 3; a++) nfp[a] = nf[a];
            prev = j;
        }
        if (out->tri_path)
            for (int b = N; b < bmax; b++) out->tri_path[r * bmax + b] = -1;
        if (N >= 1) flags |= ORC_F_VALID;
        if (N == bmax && (opts & ORC_DROP_TRAPPED)) {
            float t;
            queries++;
            int32_t j = (opts & ORC_USE_BVH) ? closest_bvh(m, o, d, prev, &t, &cnt)
                                             : closest_brute(m, o, d, prev, &t, &cnt, (opts & ORC_MT_ONLY) != 0);
            if (j >= 0) flags = (flags | ORC_F_TRAPPED) & ~ORC_F_VALID;
        }
        if (edge) flags |= ORC_F_EDGE;
        double D = 0.0;
        if (N >= 1) {
            float o0[3] = {o_in[3 * r], o_in[3 * r + 1], o_in[3 * r + 2]};
            if (opts & ORC_FP32_PATH) {
                const float k32[3] = {(float)k[0], (float)k[1], (float)k[2]};
                const float a = (k32[0] * o0[0] + k32[1] * o0[1]) + k32[2] * o0[2];
                const float c = (k32[0] * xl[0] + k32[1] * xl[1]) + k32[2] * xl[2];
                D = (double)((a + (float)P) + c);
            } else {
                D = (dotk(k, o0) + P) + dotk(k, xl);
            }
        }
        if (out->nb) out->nb[r] = N;
        if (out->tri_first) out->tri_first[r] = first;
        if (out->tri_last) out->tri_last[r] = (N >= 1) ? prev : -1;
        if (out->flags) out->flags[r] = flags;
        if (out->path) out->path[r] = P;
        if (out->D) out->D[r] = D;
        for (int a = 0; a < 3; a++) {
            if (out->d_last) out->d_last[3 * r + a] = dl[a];
            if (out->x_last) out->x_last[3 * r + a] = xl[a];
            if (out->eH_last) out->eH_last[3 * r + a] = eHl[a];
            if (out->eV_last) out->eV_last[3 * r + a] = eVl[a];
        }
        q_tot += queries;
        box_tot += cnt.box_tests;
        tri_tot += cnt.tri_tests;
        edge_tot += edge;
    }
    out->counters[0] = q_tot;
    out->counters[1] = box_tot;
    out->counters[2] = tri_tot;
    out->counters[3] = edge_tot;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Physical-optics ray-tube sum                                              */
/* ------------------------------------------------------------------------ */

/* A[f][p][q] (complex, interleaved re/im; p = receive, q = transmit, index
 * 0 = H = phi_hat, 1 = V = theta_hat) for every frequency, summed over the
 * valid rays in ray order.
 *
 * Both modes are written A = -j (k dA / 2 pi) * sum_i w_i exp(-j k D_i):
 *  PAPER  (Eq. po_sum with Gamma = -1): w = (n0 . -k) (-1)^(N+1) on the
 *         co-polar terms, 0 on the cross-polar ones; n0 is the facing normal
 *         at the first hit.
 *  VECTOR (Eqs. em5-em6 over the tube footprint dA / c_L on the last facet):
 *         J_q = d (n.e_q) - e_q (n.d) with n the facing normal, d and e_q the
 *         direction and transmit-q polarisation arriving at the last hit,
 *         c_L = max(-n.d, 1e-3), w_pq = (J_q . p_hat) / c_L. */
int orc_po(const orc_mesh *m, int64_t n, const int32_t *nb, const int32_t *tri_first, const int32_t *tri_last,
           const int32_t *flags, const double *D, const float *d_last, const double *eH_last,
           const double *eV_last, int mode, const double k[3], const double th_hat[3], const double ph_hat[3],
           double dA, const double *freqs, int nf, double *A)
{
    const int fp32 = (mode & ORC_FP32_PATH) != 0;
    mode &= ~ORC_FP32_PATH;
    double *S = (double *)calloc((size_t)nf * 8, sizeof(double));
    if (!S) return -4;
    const double *ph[2] = {ph_hat, th_hat};
    for (int64_t i = 0; i < n; i++) {
        if (!(flags[i] & ORC_F_VALID)) continue;
        double w[2][2];
        if (mode == 1) {
            const float *n0 = m->n + 3 * (int64_t)tri_first[i];
            double c0 = fabs(((double)n0[0] * k[0] + (double)n0[1] * k[1]) + (double)n0[2] * k[2]);
            double s = (nb[i] % 2 == 1) ? c0 : -c0;
            w[0][0] = s; w[1][1] = s; w[0][1] = 0.0; w[1][0] = 0.0;
        } else {
            const float *nn = m->n + 3 * (int64_t)tri_last[i];
            double sg = (flags[i] & ORC_F_BACK_LAST) ? -1.0 : 1.0;
            double nl[3] = {sg * nn[0], sg * nn[1], sg * nn[2]};
            double dl[3] = {d_last[3 * i], d_last[3 * i + 1], d_last[3 * i + 2]};
            double ndl = dot3d(nl, dl);
            double c = -ndl;
            if (c < 1e-3) c = 1e-3;
            for (int q = 0; q < 2; q++) {
                const double *e = (q == 0) ? eH_last + 3 * i : eV_last + 3 * i;
                double ne = dot3d(nl, e);
                double J[3];
                for (int a = 0; a < 3; a++) J[a] = dl[a] * ne - e[a] * ndl;
                for (int p = 0; p < 2; p++) w[p][q] = dot3d(J, ph[p]) / c;
            }
        }
        for (int f = 0; f < nf; f++) {
            double kf = 2.0 * ORC_PI * freqs[f] / ORC_C0;
            double phs = fp32 ? (double)((float)kf * (float)D[i]) : kf * D[i];
            double cr = cos(phs), si = sin(phs);
            for (int p = 0; p < 2; p++)
                for (int q = 0; q < 2; q++) {
                    double *s = S + f * 8 + (p * 2 + q) * 2;
                    /* -j * w * (cos - j sin) = w * (-sin - j cos) */
                    s[0] += -w[p][q] * si;
                    s[1] += -w[p][q] * cr;
                }
        }
    }
    for (int f = 0; f < nf; f++) {
        double kf = 2.0 * ORC_PI * freqs[f] / ORC_C0;
        double scale = kf * dA / (2.0 * ORC_PI);
        for (int e = 0; e < 8; e++) A[f * 8 + e] = scale * S[f * 8 + e];
    }
    free(S);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
