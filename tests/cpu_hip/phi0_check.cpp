// The library's phi0 (its device header, built for the host over the HIP emulation) against
// the oracle's, bit for bit, on random ellipsoids and points.  Test infrastructure only.
#include "hip/hip_runtime.h"
#include "rmx_device.h"
#include <cstdio>
#include <cstring>
#include <random>
typedef struct { int32_t kind; double centre[3]; double semi[3]; double rot[9]; } orc_shape;
extern "C" double orc_phi0(const orc_shape* s, double x, double y, double z);
int main(int argc, char** argv) {
    const long n = argc > 1 ? atol(argv[1]) : 1000000;
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::normal_distribution<double> N(0.0, 1.0);
    long bad = 0;
    for (long i = 0; i < n; ++i) {
        orc_shape o{};
        o.kind = 2;
        for (int a = 0; a < 3; ++a) { o.centre[a] = U(g) - 0.5; o.semi[a] = 0.02 + 0.38 * U(g); }
        if (i % 7 == 0) o.semi[1] = o.semi[0];               // equal axes
        double q[4]; double qn = 0; for (double& v : q) { v = N(g); qn += v * v; }
        qn = std::sqrt(qn); for (double& v : q) v /= qn;
        const double w = q[0], x = q[1], y = q[2], z = q[3];
        const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                             2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                             2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
        const bool axis = i % 5 == 0;
        for (int k = 0; k < 9; ++k) o.rot[k] = axis ? (k % 4 == 0 ? 1.0 : 0.0) : R[k];
        double v[3];
        const double scale = std::pow(10.0, -3.0 + 3.5 * U(g));
        for (int a = 0; a < 3; ++a) v[a] = o.centre[a] + scale * N(g) * o.semi[a] * 3.0;
        if (axis && i % 3 == 0) { const int a = (int)(U(g) * 3); v[a] = o.centre[a]; }
        rmx::dev::ShapeR s;
        s.kind = 2;
        s.c0 = o.centre[0]; s.c1 = o.centre[1]; s.c2 = o.centre[2];
        s.e0 = o.semi[0]; s.e1 = o.semi[1]; s.e2 = o.semi[2];
        s.r00 = o.rot[0]; s.r01 = o.rot[1]; s.r02 = o.rot[2];
        s.r10 = o.rot[3]; s.r11 = o.rot[4]; s.r12 = o.rot[5];
        s.r20 = o.rot[6]; s.r21 = o.rot[7]; s.r22 = o.rot[8];
        const double a = rmx::dev::phi0(s, v[0], v[1], v[2]);
        const double b = orc_phi0(&o, v[0], v[1], v[2]);
        if (std::memcmp(&a, &b, 8)) { if (bad < 5) printf("mismatch %.17g %.17g\n", a, b); ++bad; }
    }
    printf("phi0_check: %ld points, %ld mismatches\n", n, bad);
    return bad != 0;
}
