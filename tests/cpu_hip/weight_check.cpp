// The blur weight's certified shortcuts (rmx_weight.h, built for the host over the HIP
// emulation) against the weight from the oracle's exact distance, bit for bit, on random
// ellipsoids and points crowded around the surface band |phi0| <= 3 eps, where the
// certificates must either decide exactly or fall through.  Test infrastructure only.
#include "hip/hip_runtime.h"
#include "rmx_weight.h"
#include <cstdio>
#include <cstring>
#include <random>
typedef struct { int32_t kind; double centre[3]; double semi[3]; double rot[9]; } orc_shape;
extern "C" double orc_phi0(const orc_shape* s, double x, double y, double z);
int main(int argc, char** argv) {
    const long n = argc > 1 ? atol(argv[1]) : 1000000;
    std::mt19937_64 g(11);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::normal_distribution<double> N(0.0, 1.0);
    long bad = 0, decided = 0, tight = 0;
    for (long i = 0; i < n; ++i) {
        orc_shape o{};
        o.kind = 2;
        for (int a = 0; a < 3; ++a) { o.centre[a] = U(g) - 0.5; o.semi[a] = 0.02 + 0.38 * U(g); }
        if (i % 7 == 0) o.semi[2] = o.semi[0];               // equal axes
        double q[4]; double qn = 0; for (double& v : q) { v = N(g); qn += v * v; }
        qn = std::sqrt(qn); for (double& v : q) v /= qn;
        const double w = q[0], x = q[1], y = q[2], z = q[3];
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                             2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                             2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
        const bool axis = i % 5 == 0;
        for (int k = 0; k < 9; ++k) o.rot[k] = axis ? (k % 4 == 0 ? 1.0 : 0.0) : R[k];
        const double amin = std::fmin(o.semi[0], std::fmin(o.semi[1], o.semi[2]));
        const double eps = amin * std::pow(10.0, -3.0 + 2.7 * U(g));
        // a point of the surface along a random body direction, moved along the outward
        // normal there by t in [-3 eps, 3 eps] (or, one case in eight, anywhere nearby)
        double u[3], p[3], nb[3], yb[3];
        double s2 = 0.0;
        for (int a = 0; a < 3; ++a) { u[a] = N(g); s2 += (u[a] / o.semi[a]) * (u[a] / o.semi[a]); }
        double nn = 0.0;
        for (int a = 0; a < 3; ++a) {
            p[a] = u[a] / std::sqrt(s2);
            nb[a] = p[a] / (o.semi[a] * o.semi[a]);
            nn += nb[a] * nb[a];
        }
        const double t = (i % 8 == 0) ? amin * 4.0 * (U(g) - 0.5) : eps * 6.0 * (U(g) - 0.5);
        for (int a = 0; a < 3; ++a) yb[a] = p[a] + t * nb[a] / std::sqrt(nn);
        if (axis && i % 3 == 0) yb[(int)(U(g) * 3)] = 0.0;
        double v[3];   // world point: centre + rot * yb (body coordinates y = rot^T (v - c))
        for (int a = 0; a < 3; ++a)
            v[a] = o.centre[a] + (o.rot[3 * a] * yb[0] + o.rot[3 * a + 1] * yb[1]) +
                   o.rot[3 * a + 2] * yb[2];
        rmx::dev::ShapeR s;
        s.kind = 2;
        s.c0 = o.centre[0]; s.c1 = o.centre[1]; s.c2 = o.centre[2];
        s.e0 = o.semi[0]; s.e1 = o.semi[1]; s.e2 = o.semi[2];
        s.r00 = o.rot[0]; s.r01 = o.rot[1]; s.r02 = o.rot[2];
        s.r10 = o.rot[3]; s.r11 = o.rot[4]; s.r12 = o.rot[5];
        s.r20 = o.rot[6]; s.r21 = o.rot[7]; s.r22 = o.rot[8];
        const double got = rmx::dev::weight_at(s, v[0], v[1], v[2], eps);
        const double ph = orc_phi0(&o, v[0], v[1], v[2]);
        const double want = 1.0 - rmx::dev::heaviside_eps(ph, eps);
        if (std::memcmp(&got, &want, 8)) {
            if (bad < 5) printf("mismatch %.17g %.17g phi %.17g eps %.17g\n", got, want, ph, eps);
            ++bad;
        }
        if (got == 0.0 || got == 1.0) {
            ++decided;
            if (std::fabs(ph) < 1.25 * eps) ++tight;
        }
    }
    printf("weight_check: %ld points, %ld mismatches, %ld decided, %ld within 1.25 eps\n", n,
           bad, decided, tight);
    return bad != 0;
}
