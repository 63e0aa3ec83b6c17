// The weight of a solid in the blur zone (Lin, Derr & Rycroft, arXiv 2104.00095, main
// text eq. (sm_heavi) and eq. (mod_heaviside)): 1 - H_eps(phi0(x)), with the smoothed
// Heaviside of half-width eps.  Device code; the host test of the certificates compiles it
// over the HIP emulation.
#pragma once
#include "rmx_device.h"

namespace rmx {
namespace dev {

constexpr double kPi = 3.141592653589793;

__device__ __forceinline__ double heaviside_eps(double phi, double eps) {
    if (phi <= -eps) return 0.0;
    if (phi >= eps) return 1.0;
    return 0.5 * ((1.0 + phi / eps) + sin(kPi * phi / eps) / kPi);
}

// 1 - H_eps(phi0(x)), the weight of a solid at x.  Where the distance from x to an
// ellipsoid's surface is certainly at least eps, H_eps is exactly 0 or 1 whatever the exact
// phi0, and the bisection of the exact distance is skipped.  Three certificates, in body
// coordinates y with semi-axes a and r = eps (1 + 1e-9):
//  - with F = sum_i (y_i / a_i)^2 and g = |(y_i / a_i^2)|, the quadratic form over the ball
//    |v| <= r stays below F + 2 r g + r^2 / a_min^2 and above F - 2 r g (Cauchy-Schwarz on
//    its linear term), so the ball lies inside if the first is < 1 and outside if the
//    second is > 1;
//  - the cube |v_i| <= r around y, which holds that ball, lies outside the ellipsoid if
//    sum_i (max(|y_i| - r, 0) / a_i)^2 > 1 (the quadratic form grows with every |y_i|);
//  - with rho = |y / a|, the distance is at least (rho - 1) a_min outside (rho E contains the
//    ellipsoid grown by a ball of that radius) and (1 - rho) a_min inside.
// Each sum is compared with 1 -+ 1e-12 and each bound with r: margins far above the
// rounding of these few operations and of any exact distance.
__device__ __forceinline__ double weight_at(const ShapeR& s, double x0, double x1, double x2,
                                           double eps) {
#pragma clang fp contract(off)
    if (s.kind == 2 && finite3(x0, x1, x2)) {
        double y0, y1, y2;
        body(s, x0, x1, x2, y0, y1, y2);
        const double r = eps * (1.0 + 1e-9);
        const double amin = fmin(s.e0, fmin(s.e1, s.e2));
        const double q0 = y0 / s.e0, q1 = y1 / s.e1, q2 = y2 / s.e2;
        const double F = (q0 * q0 + q1 * q1) + q2 * q2;
        const double g0 = q0 / s.e0, g1 = q1 / s.e1, g2 = q2 / s.e2;
        const double gr = 2.0 * r * sqrt((g0 * g0 + g1 * g1) + g2 * g2);
        if ((F + gr) + (r / amin) * (r / amin) < 1.0 - 1e-12) return 1.0;   // phi0 <= -eps
        if (F - gr > 1.0 + 1e-12) return 0.0;                               // phi0 >= eps
        const double u0 = fabs(y0), u1 = fabs(y1), u2 = fabs(y2);
        const double o0 = fmax(u0 - r, 0.0) / s.e0, o1 = fmax(u1 - r, 0.0) / s.e1,
                     o2 = fmax(u2 - r, 0.0) / s.e2;
        if ((o0 * o0 + o1 * o1) + o2 * o2 > 1.0 + 1e-12) return 0.0;   // phi0 >= eps
        const double rho = sqrt(F);
        const double need = r + 1e-9 * amin * (rho + 1.0);
        if ((1.0 - rho) * amin >= need) return 1.0;
        if ((rho - 1.0) * amin >= need) return 0.0;
    }
    return 1.0 - heaviside_eps(phi0(s, x0, x1, x2), eps);
}

}  // namespace dev
}  // namespace rmx
