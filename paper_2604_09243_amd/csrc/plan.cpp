// Incidence frame and aperture ray grid of one angle, Eqs. (L1)-(L3).
//
// r = (sin t cos p, sin t sin p, cos t) points at the radar; the wave travels
// along k = -r.  The aperture plane is spanned by u = phi_hat and
// v = theta_hat (u x v = k).  Eq. L1 projects the eight bounding-box corners
// on u and v, Eq. L2 widens the extents by (1 + eta), Eq. L3 sets
// N = ceil(L~ / ds).  Rays are cell centred about the projected box centre,
// launched from a plane 1% of the box diagonal in front of the nearest corner.
#include <cmath>

#include "sbr_internal.hpp"

namespace sbr {

int plan_angle(const double bbox[6], double theta_deg, double phi_deg, double ds, double eta,
               sbr_angle_plan &out)
{
    if (!(ds > 0.0) || !std::isfinite(ds) || !std::isfinite(theta_deg) || !std::isfinite(phi_deg) ||
        !std::isfinite(eta))
        return fail(SBR_ERR_INVALID_ARG, "plan_angle: invalid ds, angle or eta");
    const double th = theta_deg * (kPi / 180.0);
    const double ph = phi_deg * (kPi / 180.0);
    const double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
    double *k = out.k_hat, *t = out.theta_hat, *p = out.phi_hat;
    k[0] = -(st * cp);
    k[1] = -(st * sp);
    k[2] = -ct;
    t[0] = ct * cp;
    t[1] = ct * sp;
    t[2] = -st;
    p[0] = -sp;
    p[1] = cp;
    p[2] = 0.0;

    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, kmin = INFINITY;
    for (int c = 0; c < 8; ++c) {
        const double x = bbox[(c & 1) ? 3 : 0];
        const double y = bbox[(c & 2) ? 4 : 1];
        const double z = bbox[(c & 4) ? 5 : 2];
        const double pu = (x * p[0] + y * p[1]) + z * p[2];
        const double pv = (x * t[0] + y * t[1]) + z * t[2];
        const double pk = (x * k[0] + y * k[1]) + z * k[2];
        umin = std::fmin(umin, pu);
        umax = std::fmax(umax, pu);
        vmin = std::fmin(vmin, pv);
        vmax = std::fmax(vmax, pv);
        kmin = std::fmin(kmin, pk);
    }
    const double lu = (1.0 + eta) * (umax - umin);
    const double lv = (1.0 + eta) * (vmax - vmin);
    const double nu = std::ceil(lu / ds), nv = std::ceil(lv / ds);
    if (!(nu < 2147483647.0) || !(nv < 2147483647.0))
        return fail(SBR_ERR_OVERFLOW, "plan_angle: ray grid too large");
    out.nu = nu < 1.0 ? 1 : static_cast<int64_t>(nu);
    out.nv = nv < 1.0 ? 1 : static_cast<int64_t>(nv);
    out.uc = 0.5 * (umin + umax);
    out.vc = 0.5 * (vmin + vmax);
    const double ex = bbox[3] - bbox[0], ey = bbox[4] - bbox[1], ez = bbox[5] - bbox[2];
    out.s0 = kmin - 0.01 * std::sqrt((ex * ex + ey * ey) + ez * ez);
    out.ds = ds;
    return SBR_OK;
}

}  // namespace sbr
