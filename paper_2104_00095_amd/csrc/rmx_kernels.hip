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

// Spread the low 4 bits of x to the low bit of 4 bytes (bit q -> byte q).  The partial
// products of x * (1 + 2^7 + 2^14 + 2^21) land on distinct bit positions, so no carries.
__device__ __forceinline__ uint32_t spread4(uint32_t x) {
    return (x * 0x00204081u) & 0x01010101u;
}

__device__ __forceinline__ unsigned long long spread8(uint32_t x) {
    return (unsigned long long)spread4(x & 15u) |
           ((unsigned long long)spread4((x >> 4) & 15u) << 32);
}

// ------------------------------------------------------------------------------------
// Classification.  A block owns a chunk of kChunkWords consecutive mask words of one
// solid; each wave streams 16 consecutive 64-cell row segments, 8 at a time (24 loads of
// 512 contiguous bytes in flight per wave), ballot-packs the interior predicate and
// writes one mask word per segment.  The chunk records whether an interior cell lies
// closer than L to a box face that is no grid wall (the band would be truncated).
// ------------------------------------------------------------------------------------
constexpr int kSeg = 8;

__global__ __launch_bounds__(256) void k_classify(Batch b) {
    const int lane = threadIdx.x & 63;
    const int wave = uniform_int(threadIdx.x >> 6);
    for (int chunk = blockIdx.x; chunk < b.n_chunks; chunk += gridDim.x) {
        const int s = uniform_int(find_solid_by_chunk(b.solids, b.n_solids, chunk));
        const DevSolid* dp = b.solids + s;
        const int n0 = dp->n0, n1 = dp->n1, n2 = dp->n2, W = dp->W, L = dp->L;
        const int64_t ncell = dp->ncell;
        const double* __restrict__ xi = dp->xi;
        unsigned long long* __restrict__ mask = dp->mask;
        const bool wl0 = dp->wall_lo[0], wh0 = dp->wall_hi[0];
        const bool wl1 = dp->wall_lo[1], wh1 = dp->wall_hi[1];
        const bool wl2 = dp->wall_lo[2], wh2 = dp->wall_hi[2];
        const ShapeR sh = load_shape(dp);
        const int nwords = n1 * n2 * W;
        const int first = (chunk - dp->chunk_base) * kChunkWords + wave * (kChunkWords / 4);
        bool trunc = false;
#pragma unroll 1
        for (int it = 0; it < kChunkWords / 4; it += kSeg) {
            const int w0 = first + it;
            if (w0 >= nwords) break;
            int row = w0 / W, wx = w0 - row * W;
            double v0[kSeg], v1[kSeg], v2[kSeg];
            int rows[kSeg], xs[kSeg];
#pragma unroll
            for (int u = 0; u < kSeg; ++u) {
                const int x = wx * 64 + lane;
                rows[u] = row;
                xs[u] = x;
                v0[u] = v1[u] = v2[u] = __builtin_nan("");
                if (w0 + u < nwords && x < n0) {
                    const int64_t c = (int64_t)row * n0 + x;
                    v0[u] = __builtin_nontemporal_load(xi + c);
                    v1[u] = __builtin_nontemporal_load(xi + ncell + c);
                    v2[u] = __builtin_nontemporal_load(xi + 2 * ncell + c);
                }
                if (++wx == W) {
                    wx = 0;
                    ++row;
                }
            }
#pragma unroll
            for (int u = 0; u < kSeg; ++u) {
                const bool in = interior(sh, v0[u], v1[u], v2[u]);
                const unsigned long long m = __ballot(in);
                if (lane == 0 && w0 + u < nwords) mask[w0 + u] = m;
                if (m) {
                    const int yy = rows[u] % n1, zz = rows[u] / n1, xx = xs[u];
                    trunc |= in && ((!wl0 && xx < L) || (!wh0 && n0 - 1 - xx < L) ||
                                    (!wl1 && yy < L) || (!wh1 && n1 - 1 - yy < L) ||
                                    (!wl2 && zz < L) || (!wh2 && n2 - 1 - zz < L));
                }
            }
        }
        const int any = __syncthreads_or(trunc);
        if (threadIdx.x == 0) b.chunk_flag[chunk] = any ? 1 : 0;
    }
}

// ------------------------------------------------------------------------------------
// Labels.  One workgroup per tile of 16 (y) x 16 (z) rows x tile_w 64-cell words (x);
// thread (tj, tk) owns one row of the tile.  The region in LDS carries a halo of L rows
// in y and z and one word on each side in x where the box continues (L <= 16 < 64), so
// after L dilations through face neighbours (64-bit shifts and ORs) the tile is exact.
// The first dilation that reaches a cell is its layer.  Per tile it records the
// interior count and the cells of each layer, and lists the band cells, grouped by
// layer, in the tile's slot range.
// ------------------------------------------------------------------------------------
constexpr int kMaxTileW = 4;
constexpr int kRowsPerThread = 9;   // ceil((16 + 2 * 16)^2 / 256)

__global__ __launch_bounds__(256) void k_label(Batch b) {
    extern __shared__ unsigned long long lds[];
    __shared__ int s_wave[4];
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const int s = uniform_int(b.tile_solid[t]);
    const DevSolid* d = &b.solids[s];
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2, W = d->W, L = d->L;
    const int TW = b.tile_w;
    const int lt = t - d->tile_base;
    const int txi = lt % d->ntx;
    const int tyi = (lt / d->ntx) % d->ty;
    const int tzi = lt / (d->ntx * d->ty);
    const int wx0 = txi * TW, tw = min(TW, W - wx0);
    const int xr0 = max(0, wx0 - 1), xr1 = min(W, wx0 + tw + 1);
    const int RW = xr1 - xr0;
    const int j0 = tyi * kTileJ, k0 = tzi * kTileK;
    const int H = L;
    const int RJ = kTileJ + 2 * H, RK = kTileK + 2 * H;
    const int R = RJ * RK;
    unsigned long long* A = lds;
    unsigned long long* B = lds + (size_t)RW * R;
    const unsigned long long tail = (n0 & 63) ? ((1ull << (n0 & 63)) - 1ull) : ~0ull;
    const unsigned long long* __restrict__ mask = d->mask;

    // Region rows owned by this thread, with their position and box membership.
    int rjs[kRowsPerThread], rks[kRowsPerThread];
    bool rok[kRowsPerThread];
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
        const int rr = tid + 256 * q;
        const int rj = rr % RJ, rk = rr / RJ;
        const int jj = j0 - H + rj, kk = k0 - H + rk;
        rjs[q] = rj;
        rks[q] = rk;
        rok[q] = rr < R && jj >= 0 && jj < n1 && kk >= 0 && kk < n2;
        if (rr < R) {
            for (int w = 0; w < RW; ++w)
                A[rr * RW + w] = rok[q] ? mask[((int64_t)kk * n1 + jj) * W + xr0 + w] : 0ull;
        }
    }
    __syncthreads();

    const int tj = tid % kTileJ, tk = tid / kTileJ;
    const int jrow = j0 + tj, krow = k0 + tk;
    const bool row_ok = jrow < n1 && krow < n2;
    const int my = ((tk + H) * RJ + (tj + H)) * RW + (wx0 - xr0);
    unsigned long long prev[kMaxTileW], p0[kMaxTileW], p1[kMaxTileW], p2[kMaxTileW],
        p3[kMaxTileW], p4[kMaxTileW];
    int cnt0 = 0;
#pragma unroll
    for (int w = 0; w < kMaxTileW; ++w) {
        prev[w] = (row_ok && w < tw) ? A[my + w] : 0ull;
        p0[w] = p1[w] = p2[w] = p3[w] = p4[w] = 0ull;
        cnt0 += __popcll(prev[w]);
    }
    {
        int excl, total;
        block_scan<4>(cnt0, excl, total, s_wave);
        if (tid == 0) b.tile_cnt[t * kLT] = total;
    }
    int lstart = 0;
    const int64_t tile_slot = d->slot_base + (int64_t)lt * b.tile_cells;
    const int32_t rowbase = (krow * n1 + jrow) * n0 + wx0 * 64;

    for (int l = 1; l <= L; ++l) {
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
            const int rr = tid + 256 * q;
            if (rr < R) {
                const int rj = rjs[q], rk = rks[q];
                for (int w = 0; w < RW; ++w) {
                    const int idx = rr * RW + w;
                    const unsigned long long c = A[idx];
                    const unsigned long long left = (w > 0) ? A[idx - 1] : 0ull;
                    const unsigned long long right = (w < RW - 1) ? A[idx + 1] : 0ull;
                    unsigned long long v = c | (c << 1) | (c >> 1) | (left >> 63) | (right << 63);
                    if (rj > 0) v |= A[idx - RW];
                    if (rj < RJ - 1) v |= A[idx + RW];
                    if (rk > 0) v |= A[idx - RW * RJ];
                    if (rk < RK - 1) v |= A[idx + RW * RJ];
                    const unsigned long long vm = !rok[q] ? 0ull : (xr0 + w == W - 1 ? tail : ~0ull);
                    B[idx] = v & vm;
                }
            }
        }
        __syncthreads();
        unsigned long long* tmp = A;
        A = B;
        B = tmp;
        unsigned long long nw[kMaxTileW];
        int cnt = 0;
#pragma unroll
        for (int w = 0; w < kMaxTileW; ++w) {
            const unsigned long long dl = (row_ok && w < tw) ? A[my + w] : 0ull;
            nw[w] = dl & ~prev[w];
            prev[w] = dl;
            if (l & 1) p0[w] |= nw[w];
            if (l & 2) p1[w] |= nw[w];
            if (l & 4) p2[w] |= nw[w];
            if (l & 8) p3[w] |= nw[w];
            if (l & 16) p4[w] |= nw[w];
            cnt += __popcll(nw[w]);
        }
        int excl, total;
        block_scan<4>(cnt, excl, total, s_wave);
        int64_t pos = tile_slot + lstart + excl;
#pragma unroll
        for (int w = 0; w < kMaxTileW; ++w) {
            unsigned long long m = nw[w];
            while (m) {
                const int bit = __ffsll((long long)m) - 1;
                m &= m - 1ull;
                b.slots[pos++] = rowbase + w * 64 + bit;
            }
        }
        if (tid == 0) {
            b.tile_cnt[t * kLT + l] = total;
            b.tile_lstart[t * kLT + l] = lstart;
        }
        lstart += total;
    }
    if (tid == 0) {
        for (int l = L + 1; l <= b.Lmax; ++l) {
            b.tile_cnt[t * kLT + l] = 0;
            b.tile_lstart[t * kLT + l] = lstart;
        }
    }

    if (!row_ok) return;
    int8_t* lab0 = d->labels + ((int64_t)krow * n1 + jrow) * n0 + wx0 * 64;
    int8_t* dec0 = d->decisions ? d->decisions + ((int64_t)krow * n1 + jrow) * n0 + wx0 * 64
                                : nullptr;
#pragma unroll
    for (int w = 0; w < kMaxTileW; ++w) {
        if (w >= tw) break;
        int8_t* lab = lab0 + 64 * w;
        int8_t* dec = dec0 ? dec0 + 64 * w : nullptr;
        const int nx = min(64, n0 - (wx0 + w) * 64);
        const bool vec = ((n0 & 7) == 0) && nx == 64 &&
                         ((reinterpret_cast<uintptr_t>(lab) & 7) == 0) &&
                         (!dec || (reinterpret_cast<uintptr_t>(dec) & 7) == 0);
        if (vec) {
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const int sh8 = 8 * g;
                // label byte = layer bits where marked, 0xFF where unmarked
                unsigned long long word =
                    spread8((uint32_t)(p0[w] >> sh8) & 255u) |
                    (spread8((uint32_t)(p1[w] >> sh8) & 255u) << 1) |
                    (spread8((uint32_t)(p2[w] >> sh8) & 255u) << 2) |
                    (spread8((uint32_t)(p3[w] >> sh8) & 255u) << 3) |
                    (spread8((uint32_t)(p4[w] >> sh8) & 255u) << 4);
                word |= spread8((uint32_t)(~prev[w] >> sh8) & 255u) * 0xFFull;
                reinterpret_cast<unsigned long long*>(lab)[g] = word;
                if (dec) reinterpret_cast<unsigned long long*>(dec)[g] = 0ull;
            }
        } else {
            for (int i = 0; i < nx; ++i) {
                int v;
                if ((prev[w] >> i) & 1ull) {
                    v = (int)(((p0[w] >> i) & 1ull) | (((p1[w] >> i) & 1ull) << 1) |
                              (((p2[w] >> i) & 1ull) << 2) | (((p3[w] >> i) & 1ull) << 3) |
                              (((p4[w] >> i) & 1ull) << 4));
                } else {
                    v = -1;
                }
                lab[i] = (int8_t)v;
                if (dec) dec[i] = 0;
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// One workgroup of 1024 threads: per-layer exclusive prefix of the tile counts (all
// layers at once), the chunk->tile table that lets a band index find its tile with one
// load, and the per-solid statistics (zeroed here, then the counts as differences of the
// prefix over the solid's tile range, and the truncation flag from the chunk flags).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan(Batch b) {
    __shared__ int s_w[kLT][16];
    const int T = b.n_tiles;
    const int Lm = b.Lmax;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < b.n_solids * kStatWords; i += 1024) b.stats[i] = 0ull;
    __syncthreads();
    int carry[kLT];
#pragma unroll
    for (int l = 0; l < kLT; ++l) carry[l] = 0;
    for (int base = 0; base < T; base += 1024) {
        const int i = base + threadIdx.x;
        int v[kLT], x[kLT];
#pragma unroll
        for (int l = 0; l < kLT; ++l) {
            v[l] = (i < T && l <= Lm) ? b.tile_cnt[i * kLT + l] : 0;
            x[l] = v[l];
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
            for (int l = 0; l < kLT; ++l) {
                const int y = __shfl_up(x[l], o, 64);
                if (lane >= o) x[l] += y;
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int l = 0; l < kLT; ++l) s_w[l][wid] = x[l];
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < kLT; ++l) {
            if (l > Lm) break;
            int wb = 0, tot = 0;
            for (int q = 0; q < 16; ++q) {
                const int tq = s_w[l][q];
                if (q < wid) wb += tq;
                tot += tq;
            }
            const int off = carry[l] + wb + x[l] - v[l];
            if (i < T) {
                b.tile_off[l * (T + 1) + i] = off;
                if (l > 0) {
                    int32_t* ct = b.chunk_tile + l * b.chunk_cap;
                    for (int c = (off + kLocateChunk - 1) / kLocateChunk;
                         c * kLocateChunk < off + v[l]; ++c)
                        ct[c] = i;
                }
            }
            carry[l] += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int l = 0; l <= Lm; ++l) b.tile_off[l * (T + 1) + T] = carry[l];
    }
    // truncation flags (rare): OR of the solid's chunk flags
    for (int c = threadIdx.x; c < b.n_chunks; c += 1024) {
        if (b.chunk_flag[c]) {
            const int s = find_solid_by_chunk(b.solids, b.n_solids, c);
            atomicOr(&b.stats[(int64_t)s * kStatWords + ST_FLAGS], FLAG_TRUNCATED);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < b.n_solids; i += 1024) {
        const DevSolid* d = b.solids + i;
        for (int l = 0; l <= Lm; ++l)
            b.stats[(int64_t)i * kStatWords + l] =
                (unsigned long long)(b.tile_off[l * (T + 1) + d->tile_base + d->n_tiles] -
                                     b.tile_off[l * (T + 1) + d->tile_base]);
    }
}

// Locate band cell `g` of layer `l`: its tile, global slot, solid and linear cell index.
struct BandCell {
    int s;
    bool skip;       // the solid's band was truncated: nothing to fit
    int64_t slot;
    int32_t cell;
};

__device__ __forceinline__ BandCell locate(const Batch& b, int l, int g) {
    const int T = b.n_tiles;
    const int32_t* off = b.tile_off + l * (T + 1);
    int t = b.chunk_tile[l * b.chunk_cap + g / kLocateChunk];
    while (off[t + 1] <= g) ++t;
    BandCell r;
    r.s = b.tile_solid[t];
    const DevSolid* d = &b.solids[r.s];
    r.skip = (b.stats[(int64_t)r.s * kStatWords + ST_FLAGS] & FLAG_TRUNCATED) != 0;
    r.slot = d->slot_base + (int64_t)(t - d->tile_base) * b.tile_cells +
             b.tile_lstart[t * kLT + l] + (g - off[t]);
    r.cell = r.skip ? 0 : b.slots[r.slot];
    return r;
}

// ------------------------------------------------------------------------------------
// Normals of the band cells of layers 1..normal_layers (one thread per cell), from the
// field before any write: central differences of phi0(xi) over the face neighbours,
// one-sided with the cell itself where a neighbour is undefined or outside the box.
// The seven cells are loaded unconditionally (clamped into the box) before any use.
// ------------------------------------------------------------------------------------
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
        if (bc.skip) continue;
        const DevSolid* d = &b.solids[bc.s];
        const ShapeR sh = load_shape(d);
        const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
        const int64_t nc = d->ncell;
        const int i = bc.cell % n0, j = (bc.cell / n0) % n1, k = bc.cell / (n0 * n1);
        const double* __restrict__ f = d->xi_normal;
        // cells: e, +x, -x, +y, -y, +z, -z
        bool in[7];
        int64_t cc[7];
        in[0] = true;
        cc[0] = bc.cell;
        in[1] = i + 1 < n0; cc[1] = in[1] ? bc.cell + 1 : bc.cell;
        in[2] = i > 0;      cc[2] = in[2] ? bc.cell - 1 : bc.cell;
        in[3] = j + 1 < n1; cc[3] = in[3] ? bc.cell + n0 : bc.cell;
        in[4] = j > 0;      cc[4] = in[4] ? bc.cell - n0 : bc.cell;
        in[5] = k + 1 < n2; cc[5] = in[5] ? bc.cell + (int64_t)n0 * n1 : bc.cell;
        in[6] = k > 0;      cc[6] = in[6] ? bc.cell - (int64_t)n0 * n1 : bc.cell;
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
        double g[3];
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
        b.normals[bc.slot] = g[0];
        b.normals[b.slot_cap + bc.slot] = g[1];
        b.normals[2 * b.slot_cap + bc.slot] = g[2];
        if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0)
            atomicAdd(&b.stats[(int64_t)bc.s * kStatWords + ST_NONORMAL], 1ull);
    }
}

// ------------------------------------------------------------------------------------
// Extrapolation of one layer.  kLanes lanes per band cell (64 / kLanes cells per wave).
// ------------------------------------------------------------------------------------
constexpr int kLanes = 8;

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

template <typename T>
__device__ __forceinline__ void reduce_lanes(Moments<T>& a) {
#pragma unroll
    for (int o = kLanes / 2; o >= 1; o >>= 1) {
#pragma unroll
        for (int q = 0; q < 10; ++q) a.m[q] += __shfl_xor(a.m[q], o, kLanes);
#pragma unroll
        for (int q = 0; q < 12; ++q) a.r[q] += __shfl_xor(a.r[q], o, kLanes);
#pragma unroll
        for (int q = 0; q < 5; ++q) a.g[q] += __shfl_xor(a.g[q], o, kLanes);
    }
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
__constant__ double c_rlen[49] = {
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

struct CellCtx {
    int i, j, k, n0, n1, n2, le;
    int64_t ncell;
    const double* __restrict__ xi;
    const int8_t* __restrict__ labels;
    int32_t anchor;               // linear index of the anchor datum
    double a0, a1, a2;            // its xi
    double g0, g1, g2, rgn;       // normal (unnormalised) and 1/|g|
};

// Accumulate the moments of the eligible data within Chebyshev radius R.  The (2R+1)^2
// rows (dy, dz) of the box are dealt to the kLanes lanes of the cell; a lane walks the
// 2R+1 cells of each of its rows (contiguous in memory).  Eq. (weight):
// w = 2^-(|dx|+|dy|+|dz|), times the cosine between x_e - x_d = -d h and the normal when
// use_normal; data with (dx gx + dy gy) + dz gz >= 0 (that exact expression, no
// contraction) get weight 0.  Ineligible cells read the anchor (0 after centring) with
// weight 0, so every load is issued unconditionally.
template <typename T, int R>
__device__ __forceinline__ void gather(const CellCtx& cx, bool use_normal, int lq,
                                       Moments<T>& acc) {
    constexpr int D = 2 * R + 1;
    constexpr int ROWS = D * D;
    constexpr int RPL = (ROWS + kLanes - 1) / kLanes;
#pragma unroll 1
    for (int q = 0; q < RPL; ++q) {
        const int row = lq + kLanes * q;
        if (row >= ROWS) break;
        const int dy = row % D - R, dz = row / D - R;
        const int jj = cx.j + dy, kk = cx.k + dz;
        const bool rowin = (unsigned)jj < (unsigned)cx.n1 && (unsigned)kk < (unsigned)cx.n2;
        const int32_t rb = (kk * cx.n1 + jj) * cx.n0;
        int32_t cc[D];
        bool ok[D];
        int lab[D];
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int ii = cx.i + u - R;
            ok[u] = rowin && (unsigned)ii < (unsigned)cx.n0;
            cc[u] = ok[u] ? rb + ii : cx.anchor;
        }
#pragma unroll
        for (int u = 0; u < D; ++u) lab[u] = cx.labels[cc[u]];
        const int rowd2 = dy * dy + dz * dz;
        T w[D];
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int dx = u - R;
            bool e = ok[u] && lab[u] >= 0 && lab[u] < cx.le;
            double ww = ldexp(1.0, -(abs(dx) + abs(dy) + abs(dz)));
            if (use_normal) {
#pragma clang fp contract(off)
                const double fx = (double)dx, fy = (double)dy, fz = (double)dz;
                const double dot = (fx * cx.g0 + fy * cx.g1) + fz * cx.g2;
                e = e && (dot < 0.0);
                ww = (-dot * c_rlen[dx * dx + rowd2] * cx.rgn) * ww;
            }
            ok[u] = e;
            w[u] = e ? (T)ww : T(0);
            if (!e) cc[u] = cx.anchor;
        }
        double v[D][3];
#pragma unroll
        for (int u = 0; u < D; ++u) {
            v[u][0] = cx.xi[cc[u]];
            v[u][1] = cx.xi[cx.ncell + cc[u]];
            v[u][2] = cx.xi[2 * cx.ncell + cc[u]];
        }
        const T fy = (T)dy, fz = (T)dz;
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int dx = u - R;
            const T tw = w[u];
            const T fx = (T)dx;
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
                acc.g[0] += 1 + ((dx * dx) << 16);
                acc.g[1] += dx + ((dx * dy) << 16);
                acc.g[2] += dy + ((dx * dz) << 16);
                acc.g[3] += dz + ((dy * dy) << 16);
                acc.g[4] += (dy * dz) + ((dz * dz) << 16);
            }
        }
    }
}

// Radii other than r_s = 2 (rare: degenerate systems): the same sums, one cell at a
// time, rows dealt to the lanes as above.
template <typename T>
__device__ __forceinline__ void gather_any(const CellCtx& cx, int r, bool use_normal, int lq,
                                        Moments<T>& acc) {
    const int D = 2 * r + 1;
    for (int row = lq; row < D * D; row += kLanes) {
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
                ww = (-dot * c_rlen[dx * dx + dy * dy + dz * dz] * cx.rgn) * ww;
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

template <typename T>
__device__ __forceinline__ void gather_r(const CellCtx& cx, int r, bool use_normal, int lq,
                                         Moments<T>& acc) {
    if (r == 2)
        gather<T, 2>(cx, use_normal, lq, acc);
    else
        gather_any<T>(cx, r, use_normal, lq, acc);
}

template <typename T>
__global__ __launch_bounds__(256) void k_extrap(Batch b, int l) {
    constexpr int kCellsPerWave = 64 / kLanes;
    const int T_ = b.n_tiles;
    const int total = b.tile_off[l * (T_ + 1) + T_];
    const int lane = threadIdx.x & 63, grp = lane / kLanes, lq = lane % kLanes;
    const int wid = uniform_int(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int nwv = gridDim.x * 4;
    for (int base = wid * kCellsPerWave; base < total; base += nwv * kCellsPerWave) {
        const int gidx = base + grp;
        if (gidx >= total) continue;
        const BandCell bc = locate(b, l, gidx);
        if (bc.skip) continue;
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
        int32_t nbc[6];
        bool nin[6];
        nin[0] = cx.i > 0;          nbc[0] = nin[0] ? bc.cell - 1 : bc.cell;
        nin[1] = cx.i + 1 < cx.n0;  nbc[1] = nin[1] ? bc.cell + 1 : bc.cell;
        nin[2] = cx.j > 0;          nbc[2] = nin[2] ? bc.cell - cx.n0 : bc.cell;
        nin[3] = cx.j + 1 < cx.n1;  nbc[3] = nin[3] ? bc.cell + cx.n0 : bc.cell;
        nin[4] = cx.k > 0;          nbc[4] = nin[4] ? bc.cell - cx.n0 * cx.n1 : bc.cell;
        nin[5] = cx.k + 1 < cx.n2;  nbc[5] = nin[5] ? bc.cell + cx.n0 * cx.n1 : bc.cell;
        int nlab[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) nlab[q] = cx.labels[nbc[q]];
        cx.anchor = bc.cell;
#pragma unroll
        for (int q = 5; q >= 0; --q)
            if (nin[q] && nlab[q] >= 0 && nlab[q] < l) cx.anchor = nbc[q];
        cx.a0 = cx.xi[cx.anchor];
        cx.a1 = cx.xi[cx.ncell + cx.anchor];
        cx.a2 = cx.xi[2 * cx.ncell + cx.anchor];
        bool has_normal = false;
        cx.g0 = cx.g1 = cx.g2 = cx.rgn = 0.0;
        if (l <= b.normal_layers) {
            cx.g0 = b.normals[bc.slot];
            cx.g1 = b.normals[b.slot_cap + bc.slot];
            cx.g2 = b.normals[2 * b.slot_cap + bc.slot];
            has_normal = cx.g0 != 0.0 || cx.g1 != 0.0 || cx.g2 != 0.0;
            if (has_normal) cx.rgn = 1.0 / norm3(cx.g0, cx.g1, cx.g2);
        }
        const bool no_normal = (l <= b.normal_layers) && !has_normal;

        // Passes: radii r_s..r_max with eq. (weight), then F1 (normal factor dropped) at
        // r_max, then F2 (kernel-weighted mean) at r_max.
        int code = -1;
        double res[3] = {0.0, 0.0, 0.0};
        const int nfit = b.r_max - b.r_s + 1;
        for (int pass = 0; pass <= nfit + 1; ++pass) {
            const bool f1 = pass == nfit, f2 = pass == nfit + 1;
            if (f1 && !has_normal) continue;
            const int r = (f1 || f2) ? b.r_max : b.r_s + pass;
            Moments<T> acc;
            zero(acc);
            gather_r<T>(cx, r, has_normal && !f1 && !f2, lq, acc);
            reduce_lanes(acc);
            if (f2) {
                const double sw = (double)acc.m[0];
                res[0] = (double)acc.r[0] / sw;
                res[1] = (double)acc.r[1] / sw;
                res[2] = (double)acc.r[2] / sw;
                code = kDecF2;
                break;
            }
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
        if (lq == 0) {
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

hipError_t launch_classify(const Batch& b, hipStream_t st) {
    const int grid = b.n_chunks < 8192 ? b.n_chunks : 8192;
    hipLaunchKernelGGL(k_classify, dim3(grid), dim3(256), 0, st, b);
    return hipGetLastError();
}

size_t label_lds_bytes(int Lmax, int tile_w, int Wmax) {
    const int RJ = kTileJ + 2 * Lmax, RK = kTileK + 2 * Lmax;
    const int RW = tile_w + 2 < Wmax ? tile_w + 2 : Wmax;
    return sizeof(unsigned long long) * 2 * (size_t)RW * RJ * RK;
}

hipError_t launch_label(const Batch& b, size_t lds, hipStream_t st) {
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
    const int grid = grid_for(max_cells, 4 * (64 / kLanes), 4096);
    if (precision == 1)
        hipLaunchKernelGGL(k_extrap<float>, dim3(grid), dim3(256), 0, st, b, layer);
    else
        hipLaunchKernelGGL(k_extrap<double>, dim3(grid), dim3(256), 0, st, b, layer);
    return hipGetLastError();
}

}  // namespace rmx
