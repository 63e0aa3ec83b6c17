// HIP kernels (gfx950) of the layer-wise WLS reference-map extrapolation.
//
// Method: Lin, Derr & Rycroft (arXiv 2104.00095), section "Extrapolation of xi(x,t)" and
// SI "Weighting scheme for weighted least squares-based extrapolation", eq. (weight).
//
// Launch chain of one call (all solids of a batch at once):
//   k_classify  streams xi once (24 B/cell), one wave per 64-cell row segment; the
//               interior predicate is ballot-packed into a 1-bit-per-cell mask.
//   k_label     per 16x16-row x 64-cell tile: the mask (+ halo of L rows and one word)
//               goes to LDS and is dilated L times through face neighbours with 64-bit
//               shifts and ORs; the first dilation that reaches a cell is its layer.
//               Writes int8 labels and the tile's band cells, grouped by layer, into the
//               tile's slot range.
//   k_scan      exclusive prefix of the per-tile layer counts (one workgroup).
//   k_normal    gradient of phi0(xi) for band cells of layers <= normal_layers, from the
//               field as it is before any write.
//   k_extrap    one launch per layer, ascending; 16 lanes per band cell gather the
//               (2r+1)^3 box, build the 4x4 normal-equation moments, reduce them over the
//               16 lanes with cross-lane shuffles, decide degeneracy by an exact integer
//               determinant, solve by Cholesky in FP64 and write xi_e in place.
// The work is gather- and bandwidth-bound, with 4x4 systems per cell: no MFMA.
#include "rmx_internal.h"

namespace rmx {
namespace {

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// Distance from body point y to the ellipsoid with semi-axes e: Lagrange multiplier of
// the closest point measured from the pole of the shortest axis among the non-zero
// coordinates, bisected until the midpoint equals an end of the bracket; the off-plane
// candidate first when every shortest-axis coordinate is exactly zero.
__device__ double ellipsoid_distance(double e0, double e1, double e2, double y0, double y1,
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
    for (int it = 0; it < 4096; ++it) {
        const double sm = 0.5 * (s0 + s1);
        if (sm <= s0 || sm >= s1) break;
        double f = 0.0;
        if (u0 > 0.0) { const double t = (e0 * u0) / (sm + d0); f = f + t * t; }
        if (u1 > 0.0) { const double t = (e1 * u1) / (sm + d1); f = f + t * t; }
        if (u2 > 0.0) { const double t = (e2 * u2) / (sm + d2); f = f + t * t; }
        f = f - 1.0;
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

// Signed distance phi0(v), negative inside; the sign is the interior predicate's.
__device__ double phi0(const ShapeR& s, double v0, double v1, double v2) {
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
__device__ __forceinline__ int find_solid_by_word(const DevSolid* s, int n, int64_t w) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s[mid].word_base <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Last tile t with off[t] <= g: the tile whose layer range holds band index g.
__device__ __forceinline__ int find_tile(const int32_t* off, int T, int g) {
    int lo = 0, hi = T - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Exclusive scan of one int per thread over a 256-thread block.
__device__ __forceinline__ void block_scan256(int v, int& excl, int& total, int* s_wave) {
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
    for (int i = 0; i < 4; ++i) {
        const int t = s_wave[i];
        if (i < wid) wb += t;
        tot += t;
    }
    excl = wb + x - v;
    total = tot;
    __syncthreads();
}

// ------------------------------------------------------------------------------------
// Zero a stats block (a kernel, not a memset node, so the chain can be graph-captured).
// ------------------------------------------------------------------------------------
__global__ void k_zero(unsigned long long* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// ------------------------------------------------------------------------------------
// Classification: one 64-cell row segment per wave, UNROLL segments in flight.
// ------------------------------------------------------------------------------------
constexpr int kClassifyUnroll = 4;

__global__ __launch_bounds__(256) void k_classify(Batch b) {
    const int lane = threadIdx.x & 63;
    const int wid = uniform_int(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int nwv = gridDim.x * 4;
    int acc_s = -1;
    unsigned long long acc = 0;
    for (int64_t w0 = wid; w0 < b.total_words; w0 += (int64_t)nwv * kClassifyUnroll) {
        double v[kClassifyUnroll][3];
        int sidx[kClassifyUnroll];
        int64_t lw[kClassifyUnroll];
        int xs[kClassifyUnroll];
        bool live[kClassifyUnroll];
#pragma unroll
        for (int u = 0; u < kClassifyUnroll; ++u) {
            const int64_t w = w0 + (int64_t)u * nwv;
            live[u] = w < b.total_words;
            v[u][0] = v[u][1] = v[u][2] = __builtin_nan("");
            sidx[u] = 0;
            lw[u] = 0;
            xs[u] = 0;
            if (live[u]) {
                const int s = find_solid_by_word(b.solids, b.n_solids, w);
                const DevSolid* d = &b.solids[s];
                const int64_t l = w - d->word_base;
                const int W = d->W;
                const int64_t row = l / W;
                const int x = (int)(l - row * W) * 64 + lane;
                sidx[u] = s;
                lw[u] = l;
                xs[u] = x;
                if (x < d->n0) {
                    const int64_t c = row * d->n0 + x;
                    const double* xi = d->xi;
                    v[u][0] = __builtin_nontemporal_load(xi + c);
                    v[u][1] = __builtin_nontemporal_load(xi + d->ncell + c);
                    v[u][2] = __builtin_nontemporal_load(xi + 2 * d->ncell + c);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kClassifyUnroll; ++u) {
            if (!live[u]) continue;
            const int s = sidx[u];
            const DevSolid* d = &b.solids[s];
            const ShapeR sh = load_shape(d);
            const bool in = interior(sh, v[u][0], v[u][1], v[u][2]);
            const unsigned long long m = __ballot(in);
            if (lane == 0) d->mask[lw[u]] = m;
            // Truncation: an interior cell closer than L to a box face that is no wall.
            bool tr = false;
            if (in) {
                const int W = d->W;
                const int row = (int)(lw[u] / W);
                const int yy = row % d->n1, zz = row / d->n1, xx = xs[u];
                const int L = d->L;
                tr = (!d->wall_lo[0] && xx < L) || (!d->wall_hi[0] && d->n0 - 1 - xx < L) ||
                     (!d->wall_lo[1] && yy < L) || (!d->wall_hi[1] && d->n1 - 1 - yy < L) ||
                     (!d->wall_lo[2] && zz < L) || (!d->wall_hi[2] && d->n2 - 1 - zz < L);
            }
            const unsigned long long tm = __ballot(tr);
            if (lane == 0) {
                if (tm) atomicOr(&b.stats[(int64_t)s * kStatWords + ST_FLAGS], FLAG_TRUNCATED);
                if (s != acc_s) {
                    if (acc_s >= 0 && acc)
                        atomicAdd(&b.stats[(int64_t)acc_s * kStatWords + ST_INTERIOR], acc);
                    acc_s = s;
                    acc = 0;
                }
                acc += (unsigned long long)__popcll(m);
            }
        }
    }
    if (lane == 0 && acc_s >= 0 && acc)
        atomicAdd(&b.stats[(int64_t)acc_s * kStatWords + ST_INTERIOR], acc);
}

// ------------------------------------------------------------------------------------
// Labels.  One workgroup per tile of 16 (y) x 16 (z) rows x one 64-cell word (x); thread
// (tj, tk) owns one row segment.  The region in LDS carries a halo of L rows in y and z
// and one word on each side in x (L <= 16 < 64), so after L dilations the tile is exact.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_label(Batch b) {
    extern __shared__ unsigned long long lds[];
    __shared__ int s_wave[4];
    const int t = blockIdx.x;
    const int s = b.tile_solid[t];
    const DevSolid* d = &b.solids[s];
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2, W = d->W, L = d->L;
    const int lt = t - d->tile_base;
    const int wx = lt % W;
    const int tyi = (lt / W) % d->ty;
    const int tzi = lt / (W * d->ty);
    const int j0 = tyi * kTileJ, k0 = tzi * kTileK;
    const int H = L;
    const int RJ = kTileJ + 2 * H, RK = kTileK + 2 * H;
    const int R3 = 3 * RJ * RK;
    unsigned long long* A = lds;
    unsigned long long* B = lds + R3;
    const bool truncated = (b.stats[(int64_t)s * kStatWords + ST_FLAGS] & FLAG_TRUNCATED) != 0;
    const unsigned long long tail =
        (n0 & 63) ? ((1ull << (n0 & 63)) - 1ull) : ~0ull;

    for (int q = threadIdx.x; q < R3; q += 256) {
        const int w = q % 3, rr = q / 3;
        const int jj = j0 - H + rr % RJ, kk = k0 - H + rr / RJ;
        const int gw = wx - 1 + w;
        unsigned long long v = 0ull;
        if (jj >= 0 && jj < n1 && kk >= 0 && kk < n2 && gw >= 0 && gw < W)
            v = d->mask[((int64_t)kk * n1 + jj) * W + gw];
        A[q] = v;
    }
    __syncthreads();

    const int tj = threadIdx.x % kTileJ, tk = threadIdx.x / kTileJ;
    const int jrow = j0 + tj, krow = k0 + tk;
    const bool row_ok = jrow < n1 && krow < n2;
    const int my = ((tk + H) * RJ + (tj + H)) * 3 + 1;
    unsigned long long prev = A[my];
    unsigned long long p0 = 0, p1 = 0, p2 = 0, p3 = 0, p4 = 0;  // bit-planes of the layer
    int lstart = 0;
    const int64_t tile_slot = d->slot_base + (int64_t)lt * kTileCells;
    const int xbase = wx * 64;
    const int32_t rowbase = (krow * n1 + jrow) * n0 + xbase;

    for (int l = 1; l <= L; ++l) {
        for (int q = threadIdx.x; q < R3; q += 256) {
            const int w = q % 3, rr = q / 3;
            const int rj = rr % RJ, rk = rr / RJ;
            const unsigned long long c = A[q];
            const unsigned long long left = (w > 0) ? A[q - 1] : 0ull;
            const unsigned long long right = (w < 2) ? A[q + 1] : 0ull;
            unsigned long long v = c | (c << 1) | (c >> 1) | (left >> 63) | (right << 63);
            if (rj > 0) v |= A[q - 3];
            if (rj < RJ - 1) v |= A[q + 3];
            if (rk > 0) v |= A[q - 3 * RJ];
            if (rk < RK - 1) v |= A[q + 3 * RJ];
            const int gw = wx - 1 + w;
            const int jj = j0 - H + rj, kk = k0 - H + rk;
            unsigned long long vm = (gw == W - 1) ? tail : ~0ull;
            if (gw < 0 || gw >= W || jj < 0 || jj >= n1 || kk < 0 || kk >= n2) vm = 0ull;
            B[q] = v & vm;
        }
        __syncthreads();
        unsigned long long* tmp = A;
        A = B;
        B = tmp;
        const unsigned long long dl = A[my];
        const unsigned long long nw = row_ok ? (dl & ~prev) : 0ull;
        prev = dl;
        if (l & 1) p0 |= nw;
        if (l & 2) p1 |= nw;
        if (l & 4) p2 |= nw;
        if (l & 8) p3 |= nw;
        if (l & 16) p4 |= nw;
        const int cnt = __popcll(nw);
        int excl, total;
        block_scan256(cnt, excl, total, s_wave);
        if (cnt && !truncated) {
            int64_t pos = tile_slot + lstart + excl;
            unsigned long long m = nw;
            while (m) {
                const int bit = __ffsll((long long)m) - 1;
                m &= m - 1ull;
                b.slots[pos++] = rowbase + bit;
            }
        }
        if (threadIdx.x == 0) {
            b.tile_cnt[t * kLT + l] = truncated ? 0 : total;
            b.tile_lstart[t * kLT + l] = lstart;
            if (total) atomicAdd(&b.stats[(int64_t)s * kStatWords + l], (unsigned long long)total);
        }
        if (!truncated) lstart += total;
    }
    if (threadIdx.x == 0) {
        for (int l = L + 1; l <= b.Lmax; ++l) {
            b.tile_cnt[t * kLT + l] = 0;
            b.tile_lstart[t * kLT + l] = lstart;
        }
    }

    if (!row_ok) return;
    const int nx = min(64, n0 - xbase);
    int8_t* lab = d->labels + ((int64_t)krow * n1 + jrow) * n0 + xbase;
    int8_t* dec = d->decisions ? d->decisions + ((int64_t)krow * n1 + jrow) * n0 + xbase : nullptr;
    const bool vec = ((n0 & 7) == 0) && nx == 64 && ((reinterpret_cast<uintptr_t>(lab) & 7) == 0) &&
                     (!dec || (reinterpret_cast<uintptr_t>(dec) & 7) == 0);
    if (vec) {
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            unsigned long long word = 0ull;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = g * 8 + q;
                unsigned long long byte;
                if ((prev >> i) & 1ull) {
                    byte = ((p0 >> i) & 1ull) | (((p1 >> i) & 1ull) << 1) |
                           (((p2 >> i) & 1ull) << 2) | (((p3 >> i) & 1ull) << 3) |
                           (((p4 >> i) & 1ull) << 4);
                } else {
                    byte = 0xFFull;
                }
                word |= byte << (8 * q);
            }
            reinterpret_cast<unsigned long long*>(lab)[g] = word;
            if (dec) reinterpret_cast<unsigned long long*>(dec)[g] = 0ull;
        }
    } else {
        for (int i = 0; i < nx; ++i) {
            int v;
            if ((prev >> i) & 1ull) {
                v = (int)(((p0 >> i) & 1ull) | (((p1 >> i) & 1ull) << 1) |
                          (((p2 >> i) & 1ull) << 2) | (((p3 >> i) & 1ull) << 3) |
                          (((p4 >> i) & 1ull) << 4));
            } else {
                v = -1;
            }
            lab[i] = (int8_t)v;
            if (dec) dec[i] = 0;
        }
    }
}

// ------------------------------------------------------------------------------------
// Per-layer exclusive prefix of tile counts (one workgroup of 1024 threads).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan(Batch b) {
    __shared__ int s_w[16];
    const int T = b.n_tiles;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int l = 1; l <= b.Lmax; ++l) {
        int carry = 0;
        for (int base = 0; base < T; base += 1024) {
            const int i = base + threadIdx.x;
            const int v = i < T ? b.tile_cnt[i * kLT + l] : 0;
            int x = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (lane == 63) s_w[wid] = x;
            __syncthreads();
            int wb = 0, tot = 0;
            for (int q = 0; q < 16; ++q) {
                const int tq = s_w[q];
                if (q < wid) wb += tq;
                tot += tq;
            }
            if (i < T) b.tile_off[l * (T + 1) + i] = carry + wb + x - v;
            carry += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) b.tile_off[l * (T + 1) + T] = carry;
    }
}

// Locate band cell `g` of layer `l`: its global slot, solid and linear cell index.
struct BandCell {
    int s;
    int64_t slot;
    int32_t cell;
};

__device__ __forceinline__ BandCell locate(const Batch& b, int l, int g) {
    const int T = b.n_tiles;
    const int32_t* off = b.tile_off + l * (T + 1);
    const int t = find_tile(off, T, g);
    BandCell r;
    r.s = b.tile_solid[t];
    const DevSolid* d = &b.solids[r.s];
    r.slot = d->slot_base + (int64_t)(t - d->tile_base) * kTileCells +
             b.tile_lstart[t * kLT + l] + (g - off[t]);
    r.cell = b.slots[r.slot];
    return r;
}

// ------------------------------------------------------------------------------------
// Normals of the band cells of layers 1..normal_layers (one thread per cell).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ bool phi_at(const DevSolid* d, const ShapeR& sh, const double* f,
                                       int i, int j, int k, double& out) {
    if (i < 0 || i >= d->n0 || j < 0 || j >= d->n1 || k < 0 || k >= d->n2) return false;
    const int64_t c = ((int64_t)k * d->n1 + j) * d->n0 + i;
    const double v0 = f[c], v1 = f[d->ncell + c], v2 = f[2 * d->ncell + c];
    if (!finite3(v0, v1, v2)) return false;
    out = phi0(sh, v0, v1, v2);
    return true;
}

__global__ __launch_bounds__(256) void k_normal(Batch b) {
    const int T = b.n_tiles;
    const int NL = min(b.normal_layers, b.Lmax);
    int total = 0;
    for (int l = 1; l <= NL; ++l) total += b.tile_off[l * (T + 1) + T];
    for (int gi = blockIdx.x * blockDim.x + threadIdx.x; gi < total;
         gi += gridDim.x * blockDim.x) {
        int l = 1, gl = gi;
        for (;;) {
            const int nl = b.tile_off[l * (T + 1) + T];
            if (gl < nl) break;
            gl -= nl;
            ++l;
        }
        const BandCell bc = locate(b, l, gl);
        const DevSolid* d = &b.solids[bc.s];
        const ShapeR sh = load_shape(d);
        const int n0 = d->n0, n1 = d->n1;
        const int i = bc.cell % n0, j = (bc.cell / n0) % n1, k = bc.cell / (n0 * n1);
        const double* f = d->xi_normal;
        double pe = 0.0;
        const bool de = phi_at(d, sh, f, i, j, k, pe);
        double g[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int ip = i + (a == 0), jp = j + (a == 1), kp = k + (a == 2);
            const int im = i - (a == 0), jm = j - (a == 1), km = k - (a == 2);
            double vp = 0.0, vm = 0.0;
            const bool dp = phi_at(d, sh, f, ip, jp, kp, vp);
            const bool dm = phi_at(d, sh, f, im, jm, km, vm);
            double ga;
            if (dp && dm) ga = 0.5 * (vp - vm);
            else if (dp && de) ga = vp - pe;
            else if (dm && de) ga = pe - vm;
            else ga = 0.0;
            g[a] = ga;
        }
        b.normals[bc.slot] = g[0];
        b.normals[b.slot_cap + bc.slot] = g[1];
        b.normals[2 * b.slot_cap + bc.slot] = g[2];
        if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0)
            atomicAdd(&b.stats[(int64_t)bc.s * kStatWords + ST_NONORMAL], 1ull);
    }
}

// ------------------------------------------------------------------------------------
// Extrapolation of one layer.  16 lanes per band cell (4 cells per wave).
// ------------------------------------------------------------------------------------
template <typename T>
struct Moments {
    T m[10];   // sum w [1,d][1,d]^T: (0,0) (0,x) (0,y) (0,z) (x,x) (x,y) (x,z) (y,y) (y,z) (z,z)
    T r[12];   // sum w [1,d] v^T: rows 1, dx, dy, dz; columns the 3 components
    int g[10]; // the same moments over the positive-weight offsets, unweighted, in integers
};

template <typename T>
__device__ __forceinline__ void zero(Moments<T>& a) {
#pragma unroll
    for (int q = 0; q < 10; ++q) a.m[q] = T(0);
#pragma unroll
    for (int q = 0; q < 12; ++q) a.r[q] = T(0);
#pragma unroll
    for (int q = 0; q < 10; ++q) a.g[q] = 0;
}

template <typename T>
__device__ __forceinline__ void reduce16(Moments<T>& a) {
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) {
#pragma unroll
        for (int q = 0; q < 10; ++q) a.m[q] += __shfl_xor(a.m[q], o, 16);
#pragma unroll
        for (int q = 0; q < 12; ++q) a.r[q] += __shfl_xor(a.r[q], o, 16);
#pragma unroll
        for (int q = 0; q < 10; ++q) a.g[q] += __shfl_xor(a.g[q], o, 16);
    }
}

// Exact determinant of the integer Gram matrix of [1, d] (Laplace expansion by the 2x2
// minors of rows 0,1 and 2,3).  |entries| <= 729*16 for r <= 4, so int64 is exact.
__device__ __forceinline__ long long det_gram(const int* g) {
    const long long a0 = g[0], a1 = g[1], a2 = g[2], a3 = g[3];       // n sx sy sz
    const long long b0 = g[1], b1 = g[4], b2 = g[5], b3 = g[6];       // sx sxx sxy sxz
    const long long c0 = g[2], c1 = g[5], c2 = g[7], c3 = g[8];       // sy sxy syy syz
    const long long d0 = g[3], d1 = g[6], d2 = g[8], d3 = g[9];       // sz sxz syz szz
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

struct CellCtx {
    int i, j, k, n0, n1, n2, le;
    int64_t ncell;
    const double* xi;
    const int8_t* labels;
    int64_t anchor;               // linear index of the anchor datum
    double a0, a1, a2;            // its xi
    double g0, g1, g2, gn;        // normal (unnormalised) and its length
};

// Weight of datum offset (dx,dy,dz) per eq. (weight); returns false for weight zero.
// The sign test is the exact expression (dx gx + dy gy) + dz gz < 0 without contraction.
__device__ __forceinline__ bool weight(const CellCtx& cx, int dx, int dy, int dz,
                                       bool use_normal, double& w) {
#pragma clang fp contract(off)
    const int ad = abs(dx) + abs(dy) + abs(dz);
    const double base = ldexp(1.0, -ad);
    if (!use_normal) {
        w = base;
        return true;
    }
    const double fx = (double)dx, fy = (double)dy, fz = (double)dz;
    const double dot = (fx * cx.g0 + fy * cx.g1) + fz * cx.g2;
    if (!(dot < 0.0)) return false;
    const double dlen = sqrt((fx * fx + fy * fy) + fz * fz);
    w = (-dot / (dlen * cx.gn)) * base;
    return true;
}

constexpr int kChunk = 8;

// Accumulate the moments of the eligible data within Chebyshev radius r, lane q of 16
// taking offsets q, q+16, ...  Ineligible slots read the anchor (offset 0 after
// centring) with weight 0, so every load can be issued unconditionally.
template <typename T>
__device__ __forceinline__ void gather(const CellCtx& cx, int r, bool use_normal, int l16,
                                       Moments<T>& acc) {
    const int D = 2 * r + 1;
    const int D3 = D * D * D;
    for (int o0 = l16; o0 < D3; o0 += 16 * kChunk) {
        int64_t cc[kChunk];
        int dd[kChunk][3];
        bool ok[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int o = o0 + 16 * u;
            const int dx = o % D - r, t2 = o / D;
            const int dy = t2 % D - r, dz = t2 / D - r;
            const int ii = cx.i + dx, jj = cx.j + dy, kk = cx.k + dz;
            dd[u][0] = dx;
            dd[u][1] = dy;
            dd[u][2] = dz;
            const bool in = o < D3 && (unsigned)ii < (unsigned)cx.n0 &&
                            (unsigned)jj < (unsigned)cx.n1 && (unsigned)kk < (unsigned)cx.n2;
            cc[u] = in ? ((int64_t)kk * cx.n1 + jj) * cx.n0 + ii : cx.anchor;
            ok[u] = in;
        }
        int lab[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) lab[u] = cx.labels[cc[u]];
        double w[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            bool e = ok[u] && lab[u] >= 0 && lab[u] < cx.le;
            double ww = 0.0;
            if (e) e = weight(cx, dd[u][0], dd[u][1], dd[u][2], use_normal, ww);
            ok[u] = e;
            w[u] = e ? ww : 0.0;
            if (!e) cc[u] = cx.anchor;
        }
        double v[kChunk][3];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            v[u][0] = cx.xi[cc[u]];
            v[u][1] = cx.xi[cx.ncell + cc[u]];
            v[u][2] = cx.xi[2 * cx.ncell + cc[u]];
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const T tw = (T)w[u];
            const T fx = (T)dd[u][0], fy = (T)dd[u][1], fz = (T)dd[u][2];
            const T v0 = (T)(v[u][0] - cx.a0), v1 = (T)(v[u][1] - cx.a1),
                    v2 = (T)(v[u][2] - cx.a2);
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
            if (ok[u]) {
                const int x = dd[u][0], y = dd[u][1], z = dd[u][2];
                acc.g[0] += 1;
                acc.g[1] += x;
                acc.g[2] += y;
                acc.g[3] += z;
                acc.g[4] += x * x;
                acc.g[5] += x * y;
                acc.g[6] += x * z;
                acc.g[7] += y * y;
                acc.g[8] += y * z;
                acc.g[9] += z * z;
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_extrap(Batch b, int l) {
    const int T_ = b.n_tiles;
    const int total = b.tile_off[l * (T_ + 1) + T_];
    const int lane = threadIdx.x & 63, grp = lane >> 4, l16 = lane & 15;
    const int wid = uniform_int(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int nwv = gridDim.x * 4;
    for (int base = wid * 4; base < total; base += nwv * 4) {
        const int gidx = base + grp;
        if (gidx >= total) continue;
        const BandCell bc = locate(b, l, gidx);
        const DevSolid* d = &b.solids[bc.s];
        CellCtx cx;
        cx.n0 = d->n0;
        cx.n1 = d->n1;
        cx.n2 = d->n2;
        cx.ncell = d->ncell;
        cx.xi = d->xi;
        cx.labels = d->labels;
        cx.le = l;
        cx.i = bc.cell % cx.n0;
        cx.j = (bc.cell / cx.n0) % cx.n1;
        cx.k = bc.cell / (cx.n0 * cx.n1);
        // Anchor: first face neighbour in a lower layer (-x, +x, -y, +y, -z, +z).  One
        // exists: the neighbour the cell was labelled from.
        cx.anchor = bc.cell;
#pragma unroll
        for (int q = 5; q >= 0; --q) {
            const int a = q >> 1, sg = (q & 1) ? 1 : -1;
            const int ii = cx.i + (a == 0 ? sg : 0), jj = cx.j + (a == 1 ? sg : 0),
                      kk = cx.k + (a == 2 ? sg : 0);
            if ((unsigned)ii < (unsigned)cx.n0 && (unsigned)jj < (unsigned)cx.n1 &&
                (unsigned)kk < (unsigned)cx.n2) {
                const int64_t c = ((int64_t)kk * cx.n1 + jj) * cx.n0 + ii;
                const int lb = cx.labels[c];
                if (lb >= 0 && lb < l) cx.anchor = c;
            }
        }
        cx.a0 = cx.xi[cx.anchor];
        cx.a1 = cx.xi[cx.ncell + cx.anchor];
        cx.a2 = cx.xi[2 * cx.ncell + cx.anchor];
        bool has_normal = false;
        cx.g0 = cx.g1 = cx.g2 = cx.gn = 0.0;
        if (l <= b.normal_layers) {
            cx.g0 = b.normals[bc.slot];
            cx.g1 = b.normals[b.slot_cap + bc.slot];
            cx.g2 = b.normals[2 * b.slot_cap + bc.slot];
            has_normal = cx.g0 != 0.0 || cx.g1 != 0.0 || cx.g2 != 0.0;
            cx.gn = norm3(cx.g0, cx.g1, cx.g2);
        }
        const bool no_normal = (l <= b.normal_layers) && !has_normal;

        int code = -1;
        double res[3] = {0.0, 0.0, 0.0};
        const int npass = b.r_max - b.r_s + 2;
        for (int pass = 0; pass < npass; ++pass) {
            const bool f1 = pass == npass - 1;
            if (f1 && !has_normal) break;
            const int r = f1 ? b.r_max : b.r_s + pass;
            Moments<T> acc;
            zero(acc);
            gather<T>(cx, r, has_normal && !f1, l16, acc);
            reduce16(acc);
            if (det_gram(acc.g) > 0) {
                double M[10], Rr[12];
#pragma unroll
                for (int q = 0; q < 10; ++q) M[q] = (double)acc.m[q];
#pragma unroll
                for (int q = 0; q < 12; ++q) Rr[q] = (double)acc.r[q];
                solve_intercept(M, Rr, res);
                code = f1 ? kDecF1 : r;
                break;
            }
        }
        if (code < 0) {
            // F2: kernel-weighted mean over the eligible data at r_max.
            Moments<T> acc;
            zero(acc);
            gather<T>(cx, b.r_max, false, l16, acc);
            reduce16(acc);
            const double sw = (double)acc.m[0];
            res[0] = (double)acc.r[0] / sw;
            res[1] = (double)acc.r[1] / sw;
            res[2] = (double)acc.r[2] / sw;
            code = kDecF2;
        }
        if (l16 == 0) {
            const int64_t c = bc.cell;
            d->xi[c] = cx.a0 + res[0];
            d->xi[cx.ncell + c] = cx.a1 + res[1];
            d->xi[2 * cx.ncell + c] = cx.a2 + res[2];
            if (d->decisions) d->decisions[c] = (int8_t)(code + (no_normal ? kDecNoNormal : 0));
            unsigned long long* st = b.stats + (int64_t)bc.s * kStatWords;
            if (code == kDecF1) atomicAdd(st + ST_F1, 1ull);
            if (code == kDecF2) atomicAdd(st + ST_F2, 1ull);
            if (code == kDecF1 || code == kDecF2 || code > b.r_s) atomicAdd(st + ST_GROWN, 1ull);
        }
    }
}

}  // namespace

// ------------------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------------------
static int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_zero(unsigned long long* p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_classify(const Batch& b, hipStream_t st) {
    // 256 CUs x 8 workgroups of 4 waves; each wave keeps 4 segments (4.5 KB) in flight.
    const int grid = grid_for(b.total_words, 4 * kClassifyUnroll, 2048);
    hipLaunchKernelGGL(k_classify, dim3(grid), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_label(const Batch& b, hipStream_t st) {
    const int RJ = kTileJ + 2 * b.Lmax, RK = kTileK + 2 * b.Lmax;
    const size_t lds = sizeof(unsigned long long) * 2 * 3 * (size_t)RJ * RK;
    hipLaunchKernelGGL(k_label, dim3(b.n_tiles), dim3(256), lds, st, b);
    return hipGetLastError();
}

hipError_t launch_scan(const Batch& b, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_normal(const Batch& b, int64_t max_cells, hipStream_t st) {
    hipLaunchKernelGGL(k_normal, dim3(grid_for(max_cells, 256, 4096)), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_extrap(const Batch& b, int layer, int precision, int64_t max_cells,
                         hipStream_t st) {
    const int grid = grid_for(max_cells, 16, 4096);
    if (precision == 1)
        hipLaunchKernelGGL(k_extrap<float>, dim3(grid), dim3(256), 0, st, b, layer);
    else
        hipLaunchKernelGGL(k_extrap<double>, dim3(grid), dim3(256), 0, st, b, layer);
    return hipGetLastError();
}

}  // namespace rmx
