// Host preparation of the mesh for the device BVH.
//
// Per triangle (Sec. 4: leaves reference triangle data; the offset epsilon of
// the reflection step is a fixed fraction of the scene size):
//   e1 = v1 - v0, e2 = v2 - v0 in float32;
//   unit normal of e1 x e2 evaluated in float64, rounded to float32;
//   degenerate when half the cross-product length is below 1e-12 diag^2.
// Bounding box over the referenced vertices; eps = fl32(1e-5 * |diag|).
#include <cmath>
#include <limits>

#include "sbr_internal.hpp"

namespace sbr {

int prepare_mesh(const float *V, int64_t nv, const int32_t *T, int64_t nt, PreparedMesh &pm)
{
    for (int64_t i = 0; i < nv * 3; ++i)
        if (!std::isfinite(V[i])) return fail(SBR_ERR_INVALID_MESH, "non-finite vertex coordinate");
    for (int64_t i = 0; i < nt * 3; ++i)
        if (T[i] < 0 || T[i] >= nv) return fail(SBR_ERR_INVALID_MESH, "triangle index out of range");

    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = std::numeric_limits<double>::infinity();
        hi[a] = -std::numeric_limits<double>::infinity();
    }
    for (int64_t j = 0; j < nt * 3; ++j) {
        const float *p = V + 3 * static_cast<int64_t>(T[j]);
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::fmin(lo[a], static_cast<double>(p[a]));
            hi[a] = std::fmax(hi[a], static_cast<double>(p[a]));
        }
    }
    for (int a = 0; a < 3; ++a) {
        pm.bbox[a] = lo[a];
        pm.bbox[3 + a] = hi[a];
    }
    const double ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    pm.diag = std::sqrt((ex * ex + ey * ey) + ez * ez);
    pm.eps = static_cast<float>(1e-5 * pm.diag);
    const double area_min = 1e-12 * pm.diag * pm.diag;

    pm.v0.resize(3 * nt);
    pm.e1.resize(3 * nt);
    pm.e2.resize(3 * nt);
    pm.n.resize(3 * nt);
    pm.degen.resize(nt);
    pm.live.clear();
    pm.live.reserve(nt);
    for (int64_t j = 0; j < nt; ++j) {
        const float *p0 = V + 3 * static_cast<int64_t>(T[3 * j + 0]);
        const float *p1 = V + 3 * static_cast<int64_t>(T[3 * j + 1]);
        const float *p2 = V + 3 * static_cast<int64_t>(T[3 * j + 2]);
        float *v0 = &pm.v0[3 * j], *e1 = &pm.e1[3 * j], *e2 = &pm.e2[3 * j], *n = &pm.n[3 * j];
        for (int a = 0; a < 3; ++a) {
            v0[a] = p0[a];
            e1[a] = p1[a] - p0[a];
            e2[a] = p2[a] - p0[a];
        }
        const double ax = e1[0], ay = e1[1], az = e1[2];
        const double bx = e2[0], by = e2[1], bz = e2[2];
        const double cx = ay * bz - az * by;
        const double cy = az * bx - ax * bz;
        const double cz = ax * by - ay * bx;
        const double len = std::sqrt((cx * cx + cy * cy) + cz * cz);
        const bool degenerate = !(0.5 * len >= area_min) || !(len > 0.0);
        pm.degen[j] = degenerate ? 1 : 0;
        if (degenerate) {
            n[0] = n[1] = n[2] = 0.0f;
        } else {
            n[0] = static_cast<float>(cx / len);
            n[1] = static_cast<float>(cy / len);
            n[2] = static_cast<float>(cz / len);
            pm.live.push_back(static_cast<int32_t>(j));
        }
    }
    return SBR_OK;
}

}  // namespace sbr
