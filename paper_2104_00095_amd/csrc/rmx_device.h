// Device helpers of the launch chain (classification, labels, per-layer brick fits).
// Method: Lin, Derr & Rycroft (arXiv 2104.00095), section "Extrapolation of xi(x,t)" and
// SI "Weighting scheme for weighted least squares-based extrapolation", eq. (weight).
#pragma once
#include "rmx_internal.h"

namespace rmx {
namespace dev {

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A load through the global address space.  Pointers read from the descriptors are
// generic, and generic (flat) loads may complete out of order with LDS accesses, so the
// compiler waits for all of them at once; global loads complete in issue order, and a
// use waits only for the loads issued before it.  (The host emulation of the kernels
// defines RMX_GLOBAL_AS away.)
#ifndef RMX_GLOBAL_AS
#define RMX_GLOBAL_AS __attribute__((address_space(1)))
#endif
template <typename T>
__device__ __forceinline__ T load_global(const T* p) {
    return *(const RMX_GLOBAL_AS T*)p;
}

// ------------------------------------------------------------------------------------
// phi0 and the interior predicate.  Evaluated without contraction, in the fixed order the
// interface documents, so that the interior decision and the normal's sign test are
// bit-identical to any other implementation of the same expressions.
// ------------------------------------------------------------------------------------
struct ShapeR {
    int kind;
    double c0, c1, c2;
    double e0, e1, e2;
    double r00, r01, r02, r10, r11, r12, r20, r21, r22;  // rot[b][a]
};

__device__ __forceinline__ ShapeR load_shape(const DevSolid* d) {
    ShapeR s;
    s.kind = d->kind;
    s.c0 = d->centre[0]; s.c1 = d->centre[1]; s.c2 = d->centre[2];
    s.e0 = d->semi[0]; s.e1 = d->semi[1]; s.e2 = d->semi[2];
    s.r00 = d->rot[0]; s.r01 = d->rot[1]; s.r02 = d->rot[2];
    s.r10 = d->rot[3]; s.r11 = d->rot[4]; s.r12 = d->rot[5];
    s.r20 = d->rot[6]; s.r21 = d->rot[7]; s.r22 = d->rot[8];
    return s;
}

__device__ __forceinline__ double norm3(double a, double b, double c) {
#pragma clang fp contract(off)
    return sqrt((a * a + b * b) + c * c);
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
    return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

__device__ __forceinline__ void body(const ShapeR& s, double v0, double v1, double v2,
                                     double& y0, double& y1, double& y2) {
#pragma clang fp contract(off)
    const double d0 = v0 - s.c0, d1 = v1 - s.c1, d2 = v2 - s.c2;
    y0 = (s.r00 * d0 + s.r10 * d1) + s.r20 * d2;
    y1 = (s.r01 * d0 + s.r11 * d1) + s.r21 * d2;
    y2 = (s.r02 * d0 + s.r12 * d1) + s.r22 * d2;
}

// phi0(xi) < 0: |xi - c|^2 < R^2 (sphere) or the quadratic form < 1 (ellipsoid).
__device__ __forceinline__ bool interior(const ShapeR& s, double v0, double v1, double v2) {
#pragma clang fp contract(off)
    if (!finite3(v0, v1, v2)) return false;
    if (s.kind == 1) {
        const double dx = v0 - s.c0, dy = v1 - s.c1, dz = v2 - s.c2;
        return ((dx * dx + dy * dy) + dz * dz) < s.e0 * s.e0;
    }
    double y0, y1, y2;
    body(s, v0, v1, v2, y0, y1, y2);
    const double q0 = y0 / s.e0, q1 = y1 / s.e1, q2 = y2 / s.e2;
    return ((q0 * q0 + q1 * q1) + q2 * q2) < 1.0;
}

__device__ __forceinline__ double pick3(int i, double a, double b, double c) {
    return i == 0 ? a : (i == 1 ? b : c);
}

// |x| within [2^-200, 2^200] (false for 0, NaN and infinities).
__device__ __forceinline__ bool mid_range(double x) {
    const double a = fabs(x);
    return a >= 0x1p-200 && a <= 0x1p200;
}

// a / b, correctly rounded, for a and b of mid_range magnitude: the reciprocal refined by
// two Newton steps, then one residual correction.  These are the steps of the hardware's
// division sequence, whose scale and fix-up steps change nothing for such operands (no
// exponent near an overflow or underflow bound, quotient within 2^+-400).  Written out,
// the divisions of one bisection step no longer wait on each other for the single
// condition register that the sequence's scale and fused-multiply-add steps share.
__device__ __forceinline__ double div_mid(double a, double b) {
    const double y0 = __builtin_amdgcn_rcp(b);
    const double y1 = fma(y0, fma(-b, y0, 1.0), y0);
    const double y2 = fma(y1, fma(-b, y1, 1.0), y1);
    const double q = a * y2;
    return fma(fma(-b, q, a), y2, q);
}

// f(s) = sum over the non-zero coordinates of (c_i / (s + d_i))^2, minus 1, in the
// bisection's arithmetic.
template <bool kMid>
__device__ __forceinline__ double ell_f(double sm, double c0, double c1, double c2, double d0,
                                        double d1, double d2, bool w0, bool w1, bool w2) {
#pragma clang fp contract(off)
    double f = 0.0;
    if (kMid) {
        // all three quotients at once (a term of a zero coordinate is formed and dropped);
        // f >= +0 throughout, so adding +0 for it changes nothing
        const double t0 = div_mid(c0, sm + d0), t1 = div_mid(c1, sm + d1),
                     t2 = div_mid(c2, sm + d2);
        f = f + (w0 ? t0 * t0 : 0.0);
        f = f + (w1 ? t1 * t1 : 0.0);
        f = f + (w2 ? t2 * t2 : 0.0);
    } else {
        if (w0) { const double t = c0 / (sm + d0); f = f + t * t; }
        if (w1) { const double t = c1 / (sm + d1); f = f + t * t; }
        if (w2) { const double t = c2 / (sm + d2); f = f + t * t; }
    }
    return f - 1.0;
}

// 1/x to a few ulps: the hardware reciprocal and one Newton step.
__device__ __forceinline__ double rcp_refined(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

// Bisection of the multiplier on [s0, s1] until the midpoint equals an end of the bracket
// (or f is exactly 0, or not a number); w_i: coordinate i is non-zero.
//
// The computed f is non-increasing in s on [s0, s1]: each operation is correctly rounded
// and monotone in its operands there (s + d_i, d_i >= 0, grows with s; c_i / x with
// c_i >= 0 shrinks as x > 0 grows; t * t for t >= 0 and the sums grow with their
// operands).  So once f(a) > 0 has been computed, every midpoint sm <= a has f(sm) > 0
// and moves s0 without an evaluation; likewise sm >= b once f(b) < 0.  The midpoints, and
// so the final bracket, are those of evaluating every step.  a and b lie 2^-44 (relative)
// either side of a few Newton steps on g(s) = F(s)^(-1/2) - 1 (F = f + 1, close to
// linear in s), taken in approximate arithmetic, or 2^-24 out where the first probe
// missed; each is used only once its own f has the needed sign.
struct Bracket {
    double s0, s1;
};
template <bool kMid>
__device__ __forceinline__ Bracket ellipsoid_bisect(double c0, double c1, double c2, double d0,
                                                    double d1, double d2, bool w0, bool w1,
                                                    bool w2, double s0, double s1) {
#pragma clang fp contract(off)
    double s = s0;
    for (int k = 0; k < 6; ++k) {
        double F = 0.0, G = 0.0;   // F = sum t_i^2, G = sum t_i^2 / (s + d_i)
        if (w0) { const double y = rcp_refined(s + d0), t = c0 * y; F = F + t * t; G = G + (t * t) * y; }
        if (w1) { const double y = rcp_refined(s + d1), t = c1 * y; F = F + t * t; G = G + (t * t) * y; }
        if (w2) { const double y = rcp_refined(s + d2), t = c2 * y; F = F + t * t; G = G + (t * t) * y; }
        double r = __builtin_amdgcn_rsq(F);
        r = r * (1.5 - (0.5 * F) * (r * r));                   // F^(-1/2)
        const double step = (r - 1.0) * rcp_refined(G * (r * r * r));   // g / g'
        s = fmin(fmax(s - step, s0), s1);                      // (a NaN step leaves s0 or s1)
    }
    const double pa = fmax(s * (1.0 - 0x1p-44), s0), pb = fmin(s * (1.0 + 0x1p-44), s1);
    const double fa = ell_f<kMid>(pa, c0, c1, c2, d0, d1, d2, w0, w1, w2);
    const double fb = ell_f<kMid>(pb, c0, c1, c2, d0, d1, d2, w0, w1, w2);
    // Any point whose f is positive bounds the root from below, any with f negative from
    // above: a probe that landed on the other side of the root is a bound of the other
    // kind, and one probe 2^-24 out then looks for the missing one.  Without it such a
    // lane would evaluate every step on that side (and hold its wave there).
    double a = fa > 0.0 ? pa : -__builtin_huge_val();
    double b = fb < 0.0 ? pb : __builtin_huge_val();
    if (b == __builtin_huge_val()) {
        if (fb > 0.0) a = fmax(a, pb);
        const double pw = fmin(s * (1.0 + 0x1p-24), s1);
        if (ell_f<kMid>(pw, c0, c1, c2, d0, d1, d2, w0, w1, w2) < 0.0) b = pw;
    }
    if (a == -__builtin_huge_val()) {
        if (fa < 0.0) b = fmin(b, pa);
        const double pw = fmax(s * (1.0 - 0x1p-24), s0);
        if (ell_f<kMid>(pw, c0, c1, c2, d0, d1, d2, w0, w1, w2) > 0.0) a = pw;
    }
    for (int it = 0; it < 4096; ++it) {
        const double sm = 0.5 * (s0 + s1);
        if (sm <= s0 || sm >= s1) break;
        double f;
        if (sm <= a)
            f = 1.0;    // f(sm) >= f(a) > 0
        else if (sm >= b)
            f = -1.0;   // f(sm) <= f(b) < 0
        else
            f = ell_f<kMid>(sm, c0, c1, c2, d0, d1, d2, w0, w1, w2);
        if (f > 0.0) {
            s0 = sm;
        } else if (f < 0.0) {
            s1 = sm;
        } else {
            s0 = sm;
            s1 = sm;
            break;
        }
    }
    return {s0, s1};
}

// Distance from body point y to the ellipsoid with semi-axes e: Lagrange multiplier of
// the closest point measured from the pole of the shortest axis among the non-zero
// coordinates, bisected until the midpoint equals an end of the bracket; the off-plane
// candidate first when every shortest-axis coordinate is exactly zero.
__device__ inline double ellipsoid_distance(double e0, double e1, double e2, double y0, double y1,
                                     double y2) {
#pragma clang fp contract(off)
    const double u0 = fabs(y0), u1 = fabs(y1), u2 = fabs(y2);
    const double q0 = e0 * e0, q1 = e1 * e1, q2 = e2 * e2;
    int amin = 0;
    if (e1 < pick3(amin, e0, e1, e2)) amin = 1;
    if (e2 < pick3(amin, e0, e1, e2)) amin = 2;
    int m = -1;
    if (u0 > 0.0) m = 0;
    if (u1 > 0.0 && (m < 0 || e1 < pick3(m, e0, e1, e2))) m = 1;
    if (u2 > 0.0 && (m < 0 || e2 < pick3(m, e0, e1, e2))) m = 2;
    const double emin = pick3(amin, e0, e1, e2);
    if (m < 0) return emin;
    const double em = pick3(m, e0, e1, e2);
    const double qmin = pick3(amin, q0, q1, q2);
    if (em > emin) {
        double S = 0.0, D = 0.0;
        if (u0 > 0.0) {
            const double x = (q0 * u0) / (q0 - qmin);
            const double t = x / e0;
            S = S + t * t;
            D = D + (x - u0) * (x - u0);
        }
        if (u1 > 0.0) {
            const double x = (q1 * u1) / (q1 - qmin);
            const double t = x / e1;
            S = S + t * t;
            D = D + (x - u1) * (x - u1);
        }
        if (u2 > 0.0) {
            const double x = (q2 * u2) / (q2 - qmin);
            const double t = x / e2;
            S = S + t * t;
            D = D + (x - u2) * (x - u2);
        }
        if (S < 1.0) return sqrt(D + qmin * (1.0 - S));
    }
    const double qm = pick3(m, q0, q1, q2);
    const double d0 = q0 - qm, d1 = q1 - qm, d2 = q2 - qm;
    double sq = 0.0;
    if (u0 > 0.0) { const double p = e0 * u0; sq = sq + p * p; }
    if (u1 > 0.0) { const double p = e1 * u1; sq = sq + p * p; }
    if (u2 > 0.0) { const double p = e2 * u2; sq = sq + p * p; }
    double s0 = em * pick3(m, u0, u1, u2);
    double s1 = sqrt(sq);
    // Every midpoint lies in [s0, s1], so (rounding being monotone) every denominator
    // sm + d_i (d_i >= 0 where u_i > 0) lies between s0 + d_i and s1 + d_i.
    const double c0 = e0 * u0, c1 = e1 * u1, c2 = e2 * u2;
    const bool w0 = u0 > 0.0, w1 = u1 > 0.0, w2 = u2 > 0.0;
    const bool mid = (!w0 || (mid_range(c0) && mid_range(s0 + d0) && mid_range(s1 + d0))) &&
                     (!w1 || (mid_range(c1) && mid_range(s0 + d1) && mid_range(s1 + d1))) &&
                     (!w2 || (mid_range(c2) && mid_range(s0 + d2) && mid_range(s1 + d2)));
    const Bracket br = mid ? ellipsoid_bisect<true>(c0, c1, c2, d0, d1, d2, w0, w1, w2, s0, s1)
                           : ellipsoid_bisect<false>(c0, c1, c2, d0, d1, d2, w0, w1, w2, s0, s1);
    s0 = br.s0;
    s1 = br.s1;
    const double s = 0.5 * (s0 + s1);
    double D = 0.0;
    {
        const double x = (u0 > 0.0) ? (q0 * u0) / (s + d0) : 0.0;
        D = D + (x - u0) * (x - u0);
    }
    {
        const double x = (u1 > 0.0) ? (q1 * u1) / (s + d1) : 0.0;
        D = D + (x - u1) * (x - u1);
    }
    {
        const double x = (u2 > 0.0) ? (q2 * u2) / (s + d2) : 0.0;
        D = D + (x - u2) * (x - u2);
    }
    return sqrt(D);
}

// phi0 of a sphere: the operations of phi0's sphere branch below, without the ellipsoid
// code (whose registers a sphere-only kernel then does not hold).
__device__ __forceinline__ double phi0_sphere(const ShapeR& s, double v0, double v1, double v2) {
#pragma clang fp contract(off)
    const double dx = v0 - s.c0, dy = v1 - s.c1, dz = v2 - s.c2;
    const double dist = fabs(sqrt((dx * dx + dy * dy) + dz * dz) - s.e0);
    const bool in = finite3(v0, v1, v2) && ((dx * dx + dy * dy) + dz * dz) < s.e0 * s.e0;
    return in ? -dist : dist;
}

// Signed distance phi0(v), negative inside; the sign is the interior predicate's.
__device__ inline double phi0(const ShapeR& s, double v0, double v1, double v2) {
#pragma clang fp contract(off)
    double dist;
    if (s.kind == 1) {
        const double dx = v0 - s.c0, dy = v1 - s.c1, dz = v2 - s.c2;
        dist = fabs(sqrt((dx * dx + dy * dy) + dz * dz) - s.e0);
    } else {
        double y0, y1, y2;
        body(s, v0, v1, v2, y0, y1, y2);
        dist = ellipsoid_distance(s.e0, s.e1, s.e2, y0, y1, y2);
    }
    return interior(s, v0, v1, v2) ? -dist : dist;
}

// ------------------------------------------------------------------------------------
// Helpers.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int find_solid_by_chunk(const DevSolid* s, int n, int c) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s[mid].chunk_base <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Exclusive scan of one int per thread over a block of NW waves.
template <int NW>
__device__ __forceinline__ void block_scan(int v, int& excl, int& total, int* s_wave) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    int wb = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int t = s_wave[i];
        if (i < wid) wb += t;
        tot += t;
    }
    excl = wb + x - v;
    total = tot;
    __syncthreads();
}

// Entries [0, count) of a list, split into one contiguous range per XCD in proportion to
// its share of the grid (workgroups are dealt to the XCDs round-robin): neighbouring
// entries, whose halos overlap, are then fetched into one L2.  The calling block takes
// begin, begin + stride, ... below end.
struct XcdRange {
    int begin, end, stride;
};
__device__ __forceinline__ XcdRange xcd_range(int count) {
    const int G = gridDim.x, x = blockIdx.x % kXcds;
    int before = 0;   // blocks on the XCDs dealt before this one
    for (int y = 0; y < x; ++y) before += (G - y + kXcds - 1) / kXcds;
    const int mine = (G - x + kXcds - 1) / kXcds;   // >= 1: this block is one of them
    XcdRange r;
    r.begin = (int)((int64_t)count * before / G) + (int)blockIdx.x / kXcds;
    r.end = (int)((int64_t)count * (before + mine) / G);
    r.stride = mine;
    return r;
}

// The same value, through an identity lane move the compiler cannot see through: work
// derived from it stays where it is written instead of being hoisted out of a loop and
// kept live (spilled) across the loop body.  All lanes of each quad must be active.
__device__ __forceinline__ int opaque_lane_value(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0xE4, 0xf, 0xf, false);   // quad_perm [0,1,2,3]
}

// ------------------------------------------------------------------------------------
// Extrapolation of one layer.  A group of NL = 4, 8 or 16 aligned lanes per band cell.
// ------------------------------------------------------------------------------------

template <typename T>
struct Moments {
    T m[10];   // sum w [1,d][1,d]^T: (0,0) (0,x) (0,y) (0,z) (x,x) (x,y) (x,z) (y,y) (y,z) (z,z)
    T r[12];   // sum w [1,d] v^T: rows 1, dx, dy, dz; columns the 3 components
    int g[5];  // unweighted integer moments over the positive-weight offsets, two 16-bit
               // fields per word: (n, sxx) (sx, sxy) (sy, sxz) (sz, syy) (syz, szz)
};

template <typename T>
__device__ __forceinline__ void zero(Moments<T>& a) {
#pragma unroll
    for (int q = 0; q < 10; ++q) a.m[q] = T(0);
#pragma unroll
    for (int q = 0; q < 12; ++q) a.r[q] = T(0);
#pragma unroll
    for (int q = 0; q < 5; ++q) a.g[q] = 0;
}

// Sums over aligned groups of NL lanes (4, 8 or 16) by DPP moves within a row: swap
// neighbours, swap pairs, then mirror the half-row (8) and the row (16).  Every lane of a
// group ends with the same, commutatively formed, sum.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_v(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp_v(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}

template <int NL, int CTRL, typename T>
__device__ __forceinline__ void reduce_step(Moments<T>& a) {
#pragma unroll
    for (int q = 0; q < 10; ++q) a.m[q] += dpp_v<CTRL>(a.m[q]);
#pragma unroll
    for (int q = 0; q < 12; ++q) a.r[q] += dpp_v<CTRL>(a.r[q]);
#pragma unroll
    for (int q = 0; q < 5; ++q) a.g[q] += dpp_i<CTRL>(a.g[q]);
}

template <int NL, typename T>
__device__ __forceinline__ void reduce_lanes(Moments<T>& a) {
    static_assert(NL == 4 || NL == 8 || NL == 16, "lane group");
    reduce_step<NL, 0xB1>(a);                   // quad_perm [1,0,3,2]
    reduce_step<NL, 0x4E>(a);                   // quad_perm [2,3,0,1]
    if (NL >= 8) reduce_step<NL, 0x141>(a);     // row_half_mirror
    if (NL >= 16) reduce_step<NL, 0x140>(a);    // row_mirror
}

// Two signed 16-bit sums packed as lo + hi * 2^16 (|sums| < 2^15 for r <= 4).
__device__ __forceinline__ void unpack2(int p, long long& lo, long long& hi) {
    const int l = (int)(short)(p & 0xffff);
    lo = l;
    hi = (long long)((p - l) >> 16);
}

// Exact determinant of the integer Gram matrix of [1, d] over the positive-weight offsets
// (Laplace expansion by the 2x2 minors of rows 0,1 and rows 2,3).  For r <= 4 the entries
// are below 729 * 16 in magnitude, so every product fits in int64.
__device__ __forceinline__ long long det_gram(const int* gp) {
    long long n, sxx, sx, sxy, sy, sxz, sz, syy, syz, szz;
    unpack2(gp[0], n, sxx);
    unpack2(gp[1], sx, sxy);
    unpack2(gp[2], sy, sxz);
    unpack2(gp[3], sz, syy);
    unpack2(gp[4], syz, szz);
    const long long a0 = n, a1 = sx, a2 = sy, a3 = sz;
    const long long b0 = sx, b1 = sxx, b2 = sxy, b3 = sxz;
    const long long c0 = sy, c1 = sxy, c2 = syy, c3 = syz;
    const long long d0 = sz, d1 = sxz, d2 = syz, d3 = szz;
    const long long s0 = a0 * b1 - a1 * b0, s1 = a0 * b2 - a2 * b0, s2 = a0 * b3 - a3 * b0;
    const long long s3 = a1 * b2 - a2 * b1, s4 = a1 * b3 - a3 * b1, s5 = a2 * b3 - a3 * b2;
    const long long t5 = c2 * d3 - c3 * d2, t4 = c1 * d3 - c3 * d1, t3 = c1 * d2 - c2 * d1;
    const long long t2 = c0 * d3 - c3 * d0, t1 = c0 * d2 - c2 * d0, t0 = c0 * d1 - c1 * d0;
    return s0 * t5 - s1 * t4 + s2 * t3 + s3 * t2 - s4 * t1 + s5 * t0;
}

// Intercept of the WLS fit from the normal equations, Cholesky in FP64.
__device__ __forceinline__ void solve_intercept(const double* M, const double* Rr,
                                                double out[3]) {
    const double l00 = sqrt(M[0]);
    const double i00 = 1.0 / l00;
    const double l10 = M[1] * i00, l20 = M[2] * i00, l30 = M[3] * i00;
    const double l11 = sqrt(M[4] - l10 * l10);
    const double i11 = 1.0 / l11;
    const double l21 = (M[5] - l20 * l10) * i11, l31 = (M[6] - l30 * l10) * i11;
    const double l22 = sqrt(M[7] - l20 * l20 - l21 * l21);
    const double i22 = 1.0 / l22;
    const double l32 = (M[8] - l30 * l20 - l31 * l21) * i22;
    const double l33 = sqrt(M[9] - l30 * l30 - l31 * l31 - l32 * l32);
    const double i33 = 1.0 / l33;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double y0 = Rr[c] * i00;
        const double y1 = (Rr[3 + c] - l10 * y0) * i11;
        const double y2 = (Rr[6 + c] - l20 * y0 - l21 * y1) * i22;
        const double y3 = (Rr[9 + c] - l30 * y0 - l31 * y1 - l32 * y2) * i33;
        const double b3 = y3 * i33;
        const double b2 = (y2 - l32 * b3) * i22;
        const double b1 = (y1 - l21 * b2 - l31 * b3) * i11;
        out[c] = (y0 - l10 * b1 - l20 * b2 - l30 * b3) * i00;
    }
}

// 1 / |d| for |d|^2 = 0..48 (offsets within radius 4).
static __constant__ double c_rlen[49] = {
    0.0, 1.0, 0.70710678118654752, 0.57735026918962576, 0.5, 0.44721359549995794,
    0.40824829046386302, 0.37796447300922723, 0.35355339059327376, 0.33333333333333333,
    0.31622776601683793, 0.30151134457776362, 0.28867513459481288, 0.27735009811261456,
    0.26726124191242438, 0.25819888974716113, 0.25, 0.24253562503633297,
    0.23570226039551584, 0.22941573387056177, 0.22360679774997897, 0.21821789023599238,
    0.21320071635561044, 0.20851441405707477, 0.20412414523193151, 0.2,
    0.19611613513818404, 0.19245008972987526, 0.18898223650461362, 0.18569533817705186,
    0.18257418583505538, 0.17960530202677491, 0.17677669529663688, 0.17407765595569785,
    0.17149858514250883, 0.16903085094570331, 0.16666666666666667, 0.16439898730535729,
    0.16222142113076254, 0.16012815380508713, 0.15811388300841897, 0.15617376188860607,
    0.15430334996209191, 0.15249857033260467, 0.15075567228888181, 0.14907119849998598,
    0.14744195615489714, 0.14586499149789456, 0.14433756729740644};

// 1 / |(fx rho_0, fy rho_1, fz rho_2)| (out of line: the rare path of unequal spacings
// keeps its registers to itself).
static __device__ __noinline__ double rlen_scaled(const double* rho, double fx, double fy, double fz) {
    return 1.0 / norm3(fx * rho[0], fy * rho[1], fz * rho[2]);
}

struct CellCtx {
    int i, j, k, n0, n1, n2, le;
    int64_t ncell;
    const double* __restrict__ xi;
    const int8_t* __restrict__ labels;
    int32_t anchor;               // linear index of the anchor datum
    double a0, a1, a2;            // its xi
    double g0, g1, g2, rgn;       // normal (unnormalised) and 1/|g / rho|
    const double* rho;            // the solid's spacing ratios; null when they are equal
};

// Accumulate, from global memory, the moments of the eligible data within Chebyshev
// radius r (used for radii beyond the staged halo).  The (2r+1)^2 rows (dy, dz) of the box
// are dealt to the NL lanes of the cell.  Eq. (weight): w = 2^-(|dx|+|dy|+|dz|), times
// the cosine between x_e - x_d = -(dx rho_x, dy rho_y, dz rho_z) h and the normal when
// use_normal; data with (dx gx + dy gy) + dz gz >= 0 (that exact expression, no
// contraction) get weight 0.
template <int NL, typename T>
__device__ __forceinline__ void gather_any(const CellCtx& cx, int r, bool use_normal, int lq,
                                        Moments<T>& acc) {
    const int D = 2 * r + 1;
    for (int row = lq; row < D * D; row += NL) {
        const int dy = row % D - r, dz = row / D - r;
        const int jj = cx.j + dy, kk = cx.k + dz;
        if ((unsigned)jj >= (unsigned)cx.n1 || (unsigned)kk >= (unsigned)cx.n2) continue;
        const int32_t rb = (kk * cx.n1 + jj) * cx.n0;
        for (int dx = -r; dx <= r; ++dx) {
            const int ii = cx.i + dx;
            if ((unsigned)ii >= (unsigned)cx.n0) continue;
            const int32_t c = rb + ii;
            const int lab = cx.labels[c];
            if (lab < 0 || lab >= cx.le) continue;
            double ww = ldexp(1.0, -(abs(dx) + abs(dy) + abs(dz)));
            if (use_normal) {
#pragma clang fp contract(off)
                const double fx = (double)dx, fy = (double)dy, fz = (double)dz;
                const double dot = (fx * cx.g0 + fy * cx.g1) + fz * cx.g2;
                if (!(dot < 0.0)) continue;
                const double rl = cx.rho ? rlen_scaled(cx.rho, fx, fy, fz)
                                         : c_rlen[dx * dx + dy * dy + dz * dz];
                ww = (-dot * rl * cx.rgn) * ww;
            }
            const T tw = (T)ww;
            const T fx = (T)dx, fy = (T)dy, fz = (T)dz;
            const T v0 = (T)(cx.xi[c] - cx.a0), v1 = (T)(cx.xi[cx.ncell + c] - cx.a1),
                    v2 = (T)(cx.xi[2 * cx.ncell + c] - cx.a2);
            const T wx = tw * fx, wy = tw * fy, wz = tw * fz;
            acc.m[0] += tw;
            acc.m[1] += wx;
            acc.m[2] += wy;
            acc.m[3] += wz;
            acc.m[4] += wx * fx;
            acc.m[5] += wx * fy;
            acc.m[6] += wx * fz;
            acc.m[7] += wy * fy;
            acc.m[8] += wy * fz;
            acc.m[9] += wz * fz;
            acc.r[0] += tw * v0;
            acc.r[1] += tw * v1;
            acc.r[2] += tw * v2;
            acc.r[3] += wx * v0;
            acc.r[4] += wx * v1;
            acc.r[5] += wx * v2;
            acc.r[6] += wy * v0;
            acc.r[7] += wy * v1;
            acc.r[8] += wy * v2;
            acc.r[9] += wz * v0;
            acc.r[10] += wz * v1;
            acc.r[11] += wz * v2;
            acc.g[0] += 1 + ((dx * dx) << 16);
            acc.g[1] += dx + ((dx * dy) << 16);
            acc.g[2] += dy + ((dx * dz) << 16);
            acc.g[3] += dz + ((dy * dy) << 16);
            acc.g[4] += (dy * dz) + ((dz * dz) << 16);
        }
    }
}

// Unnormalised gradient of phi0(xi) at box cell (i, j, k) of `f` (SI, weighting scheme):
// central differences over the face neighbours where both are defined and inside the
// box, else one-sided with the cell itself (forward first), else 0.  The seven cells are
// loaded unconditionally (clamped into the box) before any use.
__device__ __forceinline__ void normal_at(const ShapeR& sh, const double* __restrict__ f,
                                          int64_t nc, int n0, int n1, int n2, int32_t cell,
                                          int i, int j, int k, double g[3]) {
    bool in[7];
    int64_t cc[7];
    in[0] = true;
    cc[0] = cell;
    in[1] = i + 1 < n0; cc[1] = in[1] ? cell + 1 : cell;
    in[2] = i > 0;      cc[2] = in[2] ? cell - 1 : cell;
    in[3] = j + 1 < n1; cc[3] = in[3] ? cell + n0 : cell;
    in[4] = j > 0;      cc[4] = in[4] ? cell - n0 : cell;
    in[5] = k + 1 < n2; cc[5] = in[5] ? cell + (int64_t)n0 * n1 : cell;
    in[6] = k > 0;      cc[6] = in[6] ? cell - (int64_t)n0 * n1 : cell;
    double x0[7], x1[7], x2[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        x0[q] = f[cc[q]];
        x1[q] = f[nc + cc[q]];
        x2[q] = f[2 * nc + cc[q]];
    }
    double ph[7];
    bool def[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        def[q] = in[q] && finite3(x0[q], x1[q], x2[q]);
        ph[q] = def[q] ? phi0(sh, x0[q], x1[q], x2[q]) : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int qp = 1 + 2 * a, qm = 2 + 2 * a;
        double ga;
        if (def[qp] && def[qm]) ga = 0.5 * (ph[qp] - ph[qm]);
        else if (def[qp] && def[0]) ga = ph[qp] - ph[0];
        else if (def[qm] && def[0]) ga = ph[0] - ph[qm];
        else ga = 0.0;
        g[a] = ga;
    }
}

}  // namespace dev
}  // namespace rmx
