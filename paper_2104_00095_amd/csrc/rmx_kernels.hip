// HIP kernels of the reference-map band extrapolation (Lin, Derr & Rycroft, arXiv
// 2104.00095, section "Extrapolation of xi(x,t)"; SI "Weighting scheme for weighted least
// squares-based extrapolation", eq. (weight)).  One call is a chain of L + 3 launches,
// each covering every solid of the batch:
//   k_classify  streams xi once (coalesced) and packs the interior predicate
//               phi0(xi) < 0 into a 1-bit mask (wave ballots); zeroes the call's counters.
//   k_label     per 16 x 16-row tile: L bit-parallel dilations in LDS, each on the rows
//               still able to reach the tile, give the layers (first dilation reaching a
//               cell = its layer), written as int8 labels; the tile counts its interior
//               and band cells, detects a band truncated by a box face, and lists the 8^3
//               bricks holding cells of each layer (64 buckets per layer).
//   k_normal    sums the tile counts per solid; copies each layer's bucketed brick list
//               into a dense list with its count; per listed brick of layers
//               1..normal_layers, evaluates phi0(xi) once per needed cell (LDS) and forms
//               the normals of the brick's cells of that layer by central differences, from
//               the field before any write.
//   k_extrap    one launch per layer, ascending: a block stages a listed brick with a
//               halo of r_s (xi and labels, 12^3 cells, one round trip) in LDS; a group
//               of 4, 8 or 16 lanes per cell of the layer (as many as keep the brick's
//               cells in one pass) gathers the (2r+1)^3 box from LDS, accumulates the 4x4
//               normal-equation moments, reduces them by DPP moves, decides degeneracy by
//               an exact integer determinant, solves by Cholesky in FP64 and writes xi_e.
// The work is bandwidth- and latency-bound, with 4x4 systems per cell: no MFMA.
#include "rmx_device.h"

namespace rmx {
namespace {
using namespace dev;

// ------------------------------------------------------------------------------------
// Classification of mask words [wb, we) of solid d by the 4 waves of the block: each wave
// streams its 4 consecutive 64-cell row segments, ballot-packs the interior predicate
// and writes one mask word per segment (the wave's words in one store).  Cells past the
// row end (x >= n0) are never interior.
//
// Sphere: the components are read in turn, each only where the decision is still open,
// which leaves it unchanged: the test is ((dx*dx + dy*dy) + dz*dz) < R*R, and in
// round-to-nearest a sum of non-negative terms is never below any of its partial sums,
// so dx*dx >= R*R, or dx*dx + dy*dy >= R*R, already means "not interior" (a non-finite
// component fails its test as well, as in the full predicate).  The running sum is all a
// lane keeps, so a wave issues each component's 4 loads at once.  Ellipsoid: the body
// coordinates need all three components, read together.
// ------------------------------------------------------------------------------------
constexpr int kWaveWords = kChunkWords / 4;   // 4 segments per wave
constexpr int kSegE = 4;                       // ellipsoid: segments per batch

__device__ __forceinline__ void classify_sphere(const DevSolid* dp, const ShapeR& sh, int wb,
                                                int we) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int n0 = dp->n0, W = dp->W;
    const int64_t ncell = dp->ncell;
    const double* __restrict__ xi = dp->xi;
    unsigned long long* __restrict__ mask = dp->mask;
    const double T = sh.e0 * sh.e0;
    const int w0 = wb + wave * kWaveWords;
    if (w0 >= we) return;
    int row = w0 / W, wx = w0 - row * W;
    int32_t c[kWaveWords];
    double p[kWaveWords];
#pragma unroll
    for (int u = 0; u < kWaveWords; ++u) {
        const int x = wx * 64 + lane;
        c[u] = (w0 + u < we && x < n0) ? row * n0 + x : -1;
        p[u] = __builtin_nan("");
        if (c[u] >= 0) p[u] = xi[c[u]];
        if (++wx == W) {
            wx = 0;
            ++row;
        }
    }
#pragma unroll
    for (int u = 0; u < kWaveWords; ++u) {
        const double dx = p[u] - sh.c0;
        p[u] = dx * dx;
    }
#pragma unroll
    for (int u = 0; u < kWaveWords; ++u) {
        double v = __builtin_nan("");
        if (p[u] < T) v = xi[ncell + c[u]];
        const double dy = v - sh.c1;
        p[u] = p[u] + dy * dy;
    }
    unsigned long long mw = 0ull;   // lane u keeps mask word u
#pragma unroll
    for (int u = 0; u < kWaveWords; ++u) {
        double v = __builtin_nan("");
        if (p[u] < T) v = xi[2 * ncell + c[u]];
        const double dz = v - sh.c2;
        const unsigned long long m = __ballot((p[u] + dz * dz) < T);
        if (lane == u) mw = m;
    }
    if (lane < kWaveWords && w0 + lane < we) mask[w0 + lane] = mw;   // one store
}

__device__ __forceinline__ void classify_ellipsoid(const DevSolid* dp, const ShapeR& sh,
                                                   int wb, int we) {
    const int lane = threadIdx.x & 63;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int n0 = dp->n0, W = dp->W;
    const int64_t ncell = dp->ncell;
    const double* __restrict__ xi = dp->xi;
    unsigned long long* __restrict__ mask = dp->mask;
    const int first = wb + wave * kWaveWords;
#pragma unroll 1
    for (int it = 0; it < kWaveWords; it += kSegE) {
        const int w0 = first + it;
        if (w0 >= we) break;
        int row = w0 / W, wx = w0 - row * W;
        double v0[kSegE], v1[kSegE], v2[kSegE];
#pragma unroll
        for (int u = 0; u < kSegE; ++u) {
            const int x = wx * 64 + lane;
            v0[u] = v1[u] = v2[u] = __builtin_nan("");
            if (w0 + u < we && x < n0) {
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
        for (int u = 0; u < kSegE; ++u) {
            const unsigned long long m = __ballot(interior(sh, v0[u], v1[u], v2[u]));
            if (lane == 0 && w0 + u < we) mask[w0 + u] = m;
        }
    }
}

__device__ __forceinline__ void classify_words(const DevSolid* dp, int wb, int we) {
    const ShapeR sh = load_shape(dp);
    if (sh.kind == 1)
        classify_sphere(dp, sh, wb, we);
    else
        classify_ellipsoid(dp, sh, wb, we);
}

// A block owns a chunk of kChunkWords mask words of one solid.  Block 0 also zeroes the
// call's statistics and brick counters, which nothing else touches before the labels.
__global__ __launch_bounds__(256) void k_classify(Batch b) {
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < b.n_solids * kStatWords; i += 256) b.stats[i] = 0ull;
        for (int i = threadIdx.x; i < kMaxLayers * kBuckets; i += 256) b.bcount[i] = 0;
        const int nctl = (int)(sizeof(BandCtl) / sizeof(int));
        for (int i = threadIdx.x; i < nctl; i += 256) reinterpret_cast<int*>(b.band)[i] = 0;
    }
    for (int chunk = blockIdx.x; chunk < b.n_chunks; chunk += gridDim.x) {
        const int s = uniform_int(find_solid_by_chunk(b.solids, b.n_solids, chunk));
        const DevSolid* dp = b.solids + s;
        const int nwords = dp->n1 * dp->n2 * dp->W;
        const int first = (chunk - dp->chunk_base) * kChunkWords;
        classify_words(dp, first, min(first + kChunkWords, nwords));
    }
}

// ------------------------------------------------------------------------------------
// Labels of one tile of 16 (y) x 16 (z) rows x tile_w 64-cell words (x), by a block of
// 512 threads: threads i and i + 256 own row (tj, tk) = (i % 16, i / 16) of the tile, the
// first the low half of its words, the second the high half (with one word, the first
// all of it).  The region in LDS carries a halo of L rows in y and z and
// one word on each side in x where the box continues (L <= 16 < 64), so after L dilations
// through face neighbours (64-bit shifts and ORs) the tile is exact; dilation l is formed
// only on the rows within L - l of the tile, the only ones later dilations read.  Counts
// go to LDS by atomics, one wave appends the tile's bricks with one round of global
// atomics for all layers, and the labels go through an LDS transpose: whole 128-byte rows
// per store instruction in full-width tiles, aligned 4-byte words elsewhere.
// ------------------------------------------------------------------------------------
constexpr int kLabelThreads = 512;
constexpr int kRowsPerThread =      // region rows per thread at most: (16 + 2 * 16)^2 rows
    ((kTileJ + 2 * kMaxLayers) * (kTileK + 2 * kMaxLayers) + kLabelThreads - 1) / kLabelThreads;

// Label bytes of the 8 cells at bits 8g..8g+7 of a row word: the layer (bit planes
// p0..p4 hold its bits) where the cell was reached, 0xFF where not.  Bit q of a plane's
// nibble goes to bit 8q + k of a 32-bit half by one product (the partial products of
// nibble * (1 + 2^7 + 2^14 + 2^21) never overlap, and the shift by the plane k is folded
// into the constants); a cell not reached has no plane bit.  NP planes are read: layers
// below 2^NP.
template <int NP>
__device__ __forceinline__ unsigned long long label_word(
    unsigned long long p0, unsigned long long p1, unsigned long long p2, unsigned long long p3,
    unsigned long long p4, unsigned long long reached, int sh8) {
    const unsigned long long pl[5] = {p0, p1, p2, p3, p4};
    uint32_t lo = 0u, hi = 0u;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const uint32_t b = (uint32_t)(pl[k] >> sh8) & 255u;
        lo |= ((b & 15u) * (0x00204081u << k)) & (0x01010101u << k);
        hi |= ((b >> 4) * (0x00204081u << k)) & (0x01010101u << k);
    }
    const uint32_t u = (uint32_t)(~reached >> sh8) & 255u;
    lo |= (((u & 15u) * 0x00204081u) & 0x01010101u) * 0xFFu;
    hi |= (((u >> 4) * 0x00204081u) & 0x01010101u) * 0xFFu;
    return ((unsigned long long)hi << 32) | lo;
}

// The sum over the wave (every lane active): DPP sums within each row of 16 lanes (every
// lane of a row ends with the row's sum), then the four rows' sums read out.
__device__ __forceinline__ int wave_sum(int v) {
    v += dpp_i<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_i<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_i<0x141>(v);   // row_half_mirror
    v += dpp_i<0x140>(v);   // row_mirror
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

template <int N>
struct IntC {
    static constexpr int value = N;
};

// Brick r of a tile's layer-l flags (r = brick row pair * 8 * MAXTW + 8 w + g).
template <int MAXTW>
__device__ __forceinline__ bool brick_flag(const unsigned int* s_bmask, int l, int r) {
    return (s_bmask[(l - 1) * 4 + r / (8 * MAXTW)] >> (r % (8 * MAXTW))) & 1u;
}

// Bytes value(r, x) of the cells of a tile (row r = tk * kTileJ + tj, column x of the nx
// from the tile's first column xs) into dst, a box array, by the whole block; quad(r, x)
// gives the four bytes x..x+3 of row r at once.  The tile's bytes form runs: one per plane
// when it spans whole box rows (its rows of a plane are contiguous), else one per row.
// Thread i takes aligned 4-byte slot i of the runs' slots: one word store where the slot
// lies inside one row of its run, byte stores at a run's ends and across two rows.
template <typename F, typename Q>
__device__ __forceinline__ void store_tile_bytes(int8_t* dst, const DevSolid* d, int xs, int nx,
                                                 int j0, int k0, F value, Q quad) {
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
    const int nj = min(kTileJ, n1 - j0), nk = min(kTileK, n2 - k0);
    const bool whole = xs == 0 && nx == n0;
    const int len = whole ? nj * n0 : nx;   // bytes per run
    const int nrun = whole ? nk : nk * nj;
    const int U = (len + 3) / 4 + 1;        // aligned slots a run touches, at most
    for (int i = threadIdx.x; i < nrun * U; i += blockDim.x) {
        const int u = i / U, slot = i - u * U;
        const int tk = whole ? u : u / nj, tj0 = whole ? 0 : u - (u / nj) * nj;
        int8_t* run = dst + ((int64_t)(k0 + tk) * n1 + (j0 + tj0)) * n0 + xs;
        const int q0 = 4 * slot - (int)(reinterpret_cast<uintptr_t>(run) & 3u);
        if (q0 >= len) continue;
        const int qs = q0 < 0 ? 0 : q0;
        const int tj = whole ? qs / n0 : 0;   // row within the run, and column
        int r = tk * kTileJ + tj0 + tj, x = qs - tj * (whole ? n0 : 0);
        if (q0 >= 0 && q0 + 4 <= len && x + 4 <= nx) {
            *reinterpret_cast<uint32_t*>(run + q0) = quad(r, x);
            continue;
        }
        for (int q = qs; q < q0 + 4 && q < len; ++q) {
            run[q] = (int8_t)value(r, x);
            if (++x == nx) {
                x = 0;
                ++r;
            }
        }
    }
}

// Labels of a tile with no layer cell: -1 everywhere (and decision 0).  Whole-width tiles
// with 16-byte aligned rows store 16-byte chunks, consecutive threads on consecutive
// chunks of a row; other tiles go through the block's word stores.
template <int MAXTW>
__device__ __forceinline__ void label_tile_empty(const DevSolid* d, int wx0, int tw, int j0,
                                                 int k0) {
    const int tid = threadIdx.x;
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
    const int xs = wx0 * 64, nx = min(64 * tw, n0 - xs);
    const bool wide = nx == 64 * MAXTW && (n0 & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(d->labels) & 15) == 0 &&
                      (!d->decisions || (reinterpret_cast<uintptr_t>(d->decisions) & 15) == 0);
    if (wide) {
        constexpr int CPR = 4 * MAXTW;   // 16-byte chunks per row
        const uint4 ones = make_uint4(~0u, ~0u, ~0u, ~0u), zero = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int h = 0; h < 256 * CPR / kLabelThreads; ++h) {
            const int c = tid + kLabelThreads * h;
            const int row = c / CPR, off = c % CPR;
            const int jj = j0 + row % kTileJ, kk = k0 + row / kTileJ;
            if (jj < n1 && kk < n2) {
                const int64_t o = ((int64_t)kk * n1 + jj) * n0 + xs + 16 * off;
                *reinterpret_cast<uint4*>(d->labels + o) = ones;
                if (d->decisions) *reinterpret_cast<uint4*>(d->decisions + o) = zero;
            }
        }
        return;
    }
    store_tile_bytes(d->labels, d, xs, nx, j0, k0, [](int, int) { return 0xFFu; },
                     [](int, int) { return 0xFFFFFFFFu; });
    if (d->decisions)
        store_tile_bytes(d->decisions, d, xs, nx, j0, k0, [](int, int) { return 0u; },
                         [](int, int) { return 0u; });
}

template <int MAXTW>
__global__ __launch_bounds__(kLabelThreads) void k_label(Batch b) {
    constexpr int FPL = 4 * 8 * MAXTW;   // brick flags per layer: 2 (y) x 2 (z) x 8 per word
    constexpr int MW = MAXTW + 2;        // region words per row at most
    constexpr int WPH = MAXTW > 1 ? MAXTW / 2 : 1;   // row words per owning thread
    HIP_DYNAMIC_SHARED(double, lds_d)
    unsigned long long* lds = reinterpret_cast<unsigned long long*>(lds_d);
    __shared__ int s_cnt[kLT];
    __shared__ int s_trunc;
    __shared__ unsigned int s_bmask[kMaxLayers * 4];   // bricks holding layer-l cells:
                                                        // [l-1][2 x 2 brick rows], bit 8w + g

    const int t = blockIdx.x;
    const int s = uniform_int(b.tile_solid[t]);
    const DevSolid* d = b.solids + s;
    unsigned long long* st = b.stats + (int64_t)s * kStatWords;
    const int tid = threadIdx.x;
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2, W = d->W, L = d->L;
    const int lt = t - d->tile_base;
    const int txi = lt % d->ntx;
    const int tyi = (lt / d->ntx) % d->ty;
    const int tzi = lt / (d->ntx * d->ty);
    const int wx0 = txi * MAXTW, tw = min(MAXTW, W - wx0);
    const int xr0 = max(0, wx0 - 1), xr1 = min(W, wx0 + tw + 1);
    const int RW = xr1 - xr0;
    const int RS = RW | 1;   // row stride in words: odd, so that rows fall on distinct banks
    const int j0 = tyi * kTileJ, k0 = tzi * kTileK;
    const int RJ = kTileJ + 2 * L, RK = kTileK + 2 * L;
    const int R = RJ * RK;
    unsigned long long* A = lds;
    unsigned long long* B = lds + (size_t)RS * R;
    const unsigned long long tail = (n0 & 63) ? ((1ull << (n0 & 63)) - 1ull) : ~0ull;
    const unsigned long long* __restrict__ mask = d->mask;

    for (int q = tid; q < L * 4; q += kLabelThreads) s_bmask[q] = 0u;
    if (tid < kLT) s_cnt[tid] = 0;
    if (tid == 0) s_trunc = 0;
    // The mask rows of the region (rows outside the box: empty).  Every load of the
    // thread is issued into registers before the first LDS store, so they overlap instead
    // of each waiting for the previous one.
    unsigned long long mv[kRowsPerThread][MW];
    unsigned long long any = 0ull;
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
        const int rr = tid + kLabelThreads * q;
        const int rj = rr % RJ, rk = rr / RJ;
        const int jj = j0 - L + rj, kk = k0 - L + rk;
        const bool ok = rr < R && jj >= 0 && jj < n1 && kk >= 0 && kk < n2;
        const int64_t base = ok ? ((int64_t)kk * n1 + jj) * W + xr0 : 0;
#pragma unroll
        for (int w = 0; w < MW; ++w) {
            mv[q][w] = (ok && w < RW) ? mask[base + w] : 0ull;
            any |= mv[q][w];
        }
    }
    // A tile whose whole region holds no interior cell has no layer cell either: its
    // labels are all -1 (decisions 0), its counts 0, and it lists no brick.
    if (!__syncthreads_or(any != 0ull)) {
        if (tid <= L) b.tile_cnt[(int64_t)t * kLT + tid] = 0;
        label_tile_empty<MAXTW>(d, wx0, tw, j0, k0);
        return;
    }
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
        const int rr = tid + kLabelThreads * q;
        if (rr < R) {
#pragma unroll
            for (int w = 0; w < MW; ++w)
                if (w < RW) A[rr * RS + w] = mv[q][w];
        }
    }
    __syncthreads();

    const int row = tid & 255, wb = (tid >> 8) * WPH;   // the row; its first owned word
    const int tj = row % kTileJ, tk = row / kTileJ;
    const int jrow = j0 + tj, krow = k0 + tk;
    const bool row_ok = jrow < n1 && krow < n2;
    const int my = ((tk + L) * RJ + (tj + L)) * RS + (wx0 - xr0) + wb;
    // owned words wb + w, w < WPH (none past the tile)
    unsigned long long prev[WPH], p0[WPH], p1[WPH], p2[WPH], p3[WPH], p4[WPH];
    int cnt0 = 0;
    bool trunc = false;
#pragma unroll
    for (int w = 0; w < WPH; ++w) {
        prev[w] = (row_ok && wb + w < tw) ? A[my + w] : 0ull;
        p0[w] = p1[w] = p2[w] = p3[w] = p4[w] = 0ull;
        cnt0 += __popcll(prev[w]);
        // An interior cell closer than L to a box face that is no grid wall: the band
        // would leave the box (reported; the solid's band is then not fitted).
        if (prev[w]) {
            const int x0 = (wx0 + wb + w) * 64;
            if (!d->wall_lo[0] && x0 < L) {
                const int nb = min(64, L - x0);
                trunc |= (prev[w] & (nb == 64 ? ~0ull : ((1ull << nb) - 1ull))) != 0ull;
            }
            if (!d->wall_hi[0] && x0 + 63 >= n0 - L) {
                const int f = max(0, n0 - L - x0);
                trunc |= (prev[w] & (~0ull << f)) != 0ull;
            }
            trunc |= (!d->wall_lo[1] && jrow < L) || (!d->wall_hi[1] && jrow >= n1 - L) ||
                     (!d->wall_lo[2] && krow < L) || (!d->wall_hi[2] && krow >= n2 - L);
        }
    }
    // counts: wave sums, then one LDS atomic per wave
    const int lane = tid & 63;
    cnt0 = wave_sum(cnt0);
    if (lane == 0 && cnt0) atomicAdd(&s_cnt[0], cnt0);
    if (trunc) s_trunc = 1;

    const int by2 = (tk >> 3) * 2 + (tj >> 3);   // which of the tile's 2 x 2 brick rows
    for (int l = 1; l <= L; ++l) {
        // One dilation step through face neighbours (or, with the 26-neighbour adjacency,
        // through every cell of the 3^3 cube), A -> B, over the rows that can still reach
        // the tile: D_l is needed only within L - l rows of it, i.e. on region rows
        // [l, RJ - l) x [l, RK - l) (their neighbours lie inside the region).  A row's own
        // words come from registers, its neighbour rows from LDS.
        const unsigned long long* __restrict__ Ar = A;
        unsigned long long* __restrict__ Br = B;
        const int SJ = RJ - 2 * l, S = SJ * (RK - 2 * l);
        for (int i = tid; i < S; i += kLabelThreads) {
            const int rk = l + i / SJ, rj = l + i % SJ;
            const int jj = j0 - L + rj, kk = k0 - L + rk;
            const bool rok = jj >= 0 && jj < n1 && kk >= 0 && kk < n2;
            const int base = (rk * RJ + rj) * RS;
            unsigned long long c[MW];
#pragma unroll
            for (int w = 0; w < MW; ++w) c[w] = w < RW ? Ar[base + w] : 0ull;
#pragma unroll
            for (int w = 0; w < MW; ++w) {
                if (w >= RW) break;
                const int idx = base + w;
                const unsigned long long left = w > 0 ? c[w - 1] : 0ull;
                const unsigned long long right = w < MW - 1 ? c[w + 1] : 0ull;
                unsigned long long v = c[w] | (c[w] << 1) | (c[w] >> 1) | (left >> 63) |
                                       (right << 63);
                if (!b.adj26) {
                    v |= Ar[idx - RS] | Ar[idx + RS] | Ar[idx - RS * RJ] | Ar[idx + RS * RJ];
                } else {
                    // cube adjacency: the x-dilated words of the eight neighbour rows
#pragma unroll
                    for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
                        for (int dj = -1; dj <= 1; ++dj) {
                            if (dj == 0 && dk == 0) continue;
                            const int q = idx + dj * RS + dk * RS * RJ;
                            const unsigned long long m = Ar[q];
                            const unsigned long long ml = w > 0 ? Ar[q - 1] : 0ull;
                            const unsigned long long mr = w + 1 < RW ? Ar[q + 1] : 0ull;
                            v |= m | (m << 1) | (m >> 1) | (ml >> 63) | (mr << 63);
                        }
                }
                const unsigned long long vm = !rok ? 0ull : (xr0 + w == W - 1 ? tail : ~0ull);
                Br[idx] = v & vm;
            }
        }
        __syncthreads();
        unsigned long long* tmp = A;
        A = B;
        B = tmp;
        int cnt = 0;
        unsigned int fl = 0u;   // bricks of this row holding a layer-l cell: bit 8w + g
#pragma unroll
        for (int w = 0; w < WPH; ++w) {
            const unsigned long long dl = (row_ok && wb + w < tw) ? A[my + w] : 0ull;
            const unsigned long long nw = dl & ~prev[w];
            prev[w] = dl;
            if (l & 1) p0[w] |= nw;
            if (l & 2) p1[w] |= nw;
            if (l & 4) p2[w] |= nw;
            if (l & 8) p3[w] |= nw;
            if (l & 16) p4[w] |= nw;
            cnt += __popcll(nw);
#pragma unroll
            for (int g = 0; g < 8; ++g)
                if ((nw >> (8 * g)) & 255ull) fl |= 1u << ((wb + w) * 8 + g);
        }
        // Wave sums of the counts; the flags ORed over the lanes of each brick row pair (a
        // wave's lanes share tk >> 3, lane bit 3 is tj >> 3): then lane 0's LDS atomics.
        cnt = wave_sum(cnt);
        fl |= dpp_i<0xB1>((int)fl);    // quad_perm [1,0,3,2]
        fl |= dpp_i<0x4E>((int)fl);    // quad_perm [2,3,0,1]
        fl |= dpp_i<0x141>((int)fl);   // row_half_mirror: the OR over each 8 lanes
        const unsigned int f0 = (unsigned)(__builtin_amdgcn_readlane((int)fl, 0) |
                                           __builtin_amdgcn_readlane((int)fl, 16) |
                                           __builtin_amdgcn_readlane((int)fl, 32) |
                                           __builtin_amdgcn_readlane((int)fl, 48));
        const unsigned int f1 = (unsigned)(__builtin_amdgcn_readlane((int)fl, 8) |
                                           __builtin_amdgcn_readlane((int)fl, 24) |
                                           __builtin_amdgcn_readlane((int)fl, 40) |
                                           __builtin_amdgcn_readlane((int)fl, 56));
        if (lane == 0) {
            if (cnt) atomicAdd(&s_cnt[l], cnt);
            if (f0) atomicOr(&s_bmask[(l - 1) * 4 + (by2 & ~1)], f0);
            if (f1) atomicOr(&s_bmask[(l - 1) * 4 + (by2 | 1)], f1);
        }
    }
    __syncthreads();   // counts, flags and the last step complete; A/B free
    if (tid <= L) b.tile_cnt[(int64_t)t * kLT + tid] = s_cnt[tid];
    if (tid == 0 && s_trunc) atomicOr(st + ST_FLAGS, FLAG_TRUNCATED);

    // Bricks holding cells of each layer, appended to the layer's list in this tile's
    // bucket: wave 0 counts every layer, reserves all layers' slots with one round of
    // atomics, then writes the entries.  A brick lies in exactly one tile, so a tile lists
    // at most FPL bricks per layer and its bucket never overflows.
    if (tid < 64) {   // (lane == tid)
        const int bk = t % kBuckets;
        const int64_t base0 = bucket_base(bk, b.n_tiles, b.tile_w);
        const int64_t cap = bucket_base(bk + 1, b.n_tiles, b.tile_w) - base0;
        int mytot = 0;   // lane l - 1: bricks of layer l
        for (int l = 1; l <= L; ++l) {
            int tot = 0;
            for (int f0 = 0; f0 < FPL; f0 += 64)
                tot += __popcll(__ballot(f0 + lane < FPL && brick_flag<MAXTW>(s_bmask, l, f0 + lane)));
            if (lane == l - 1) mytot = tot;
        }
        int mybase = 0;
        if (lane < L && mytot > 0) mybase = atomicAdd(b.bcount + lane * kBuckets + bk, mytot);
        for (int l = 1; l <= L; ++l) {
            const int lbase = __shfl(mybase, l - 1, 64);
            int run = 0;
            for (int f0 = 0; f0 < FPL; f0 += 64) {
                const int r = f0 + lane;
                const bool f = r < FPL && brick_flag<MAXTW>(s_bmask, l, r);
                const unsigned long long bal = __ballot(f);
                if (f) {
                    const int pos = lbase + run + __popcll(bal & ((1ull << lane) - 1ull));
                    const int yz = r / (8 * MAXTW), xb = r % (8 * MAXTW);
                    const int bx = wx0 * 8 + xb, by = 2 * tyi + (yz & 1), bz = 2 * tzi + (yz >> 1);
                    if (pos < cap)
                        b.blist[(int64_t)(l - 1) * b.blist_cap + base0 + pos] =
                            ((unsigned long long)s << 32) |
                            (unsigned long long)(bx | (by << 10) | (bz << 20));
                    else
                        atomicOr(st + ST_FLAGS, FLAG_OVERFLOW);
                }
                run += __popcll(bal);
            }
        }
    }

    // Labels: byte = layer where the cell was reached, 0xFF where not.  Each thread forms
    // its row's label words in LDS; full-width tiles with aligned rows then store whole
    // 128-byte rows per store instruction, other tiles go through the block's word stores.
    constexpr int TS = 8 * MAXTW + 1;   // padded row stride: rows on distinct banks
    unsigned long long* T = lds;         // [256 rows][TS] label words
    {
        // the planes the layers 1..L use (L uniform: one branch per tile)
        auto fill = [&](auto np) {
            constexpr int NP = decltype(np)::value;
#pragma unroll
            for (int w = 0; w < WPH; ++w) {
                if (wb + w >= MAXTW) break;   // (the second thread of a one-word row)
#pragma unroll
                for (int g = 0; g < 8; ++g)
                    T[row * TS + (wb + w) * 8 + g] =
                        label_word<NP>(p0[w], p1[w], p2[w], p3[w], p4[w], prev[w], 8 * g);
            }
        };
        if (L < 8)
            fill(IntC<3>{});
        else
            fill(IntC<5>{});
    }
    __syncthreads();
    const bool full = tw == MAXTW && (wx0 + MAXTW) * 64 <= n0 && (n0 & 7) == 0 &&
                      (reinterpret_cast<uintptr_t>(d->labels) & 7) == 0 &&
                      (!d->decisions || (reinterpret_cast<uintptr_t>(d->decisions) & 7) == 0);
    if (full) {   // uniform
        constexpr int CPR = 8 * MAXTW;   // 8-byte chunks per tile row
#pragma unroll
        for (int h = 0; h < 256 * CPR / kLabelThreads; ++h) {
            const int ch = tid + kLabelThreads * h;
            const int row = ch / CPR, off = ch % CPR;   // row = tk * 16 + tj
            const int rj = j0 + row % kTileJ, rk = k0 + row / kTileJ;
            if (rj < n1 && rk < n2) {
                const int64_t o = ((int64_t)rk * n1 + rj) * n0 + wx0 * 64 + 8 * off;
                reinterpret_cast<unsigned long long*>(d->labels + o)[0] = T[row * TS + off];
                if (d->decisions) reinterpret_cast<unsigned long long*>(d->decisions + o)[0] = 0ull;
            }
        }
    } else {
        const int xs = wx0 * 64, nx = min(64 * tw, n0 - xs);
        const uint8_t* Tb = reinterpret_cast<const uint8_t*>(T);
        const uint32_t* Tw = reinterpret_cast<const uint32_t*>(T);
        // four bytes of a row from the two aligned words holding them (a row's padding word
        // lies past its last byte)
        auto quad = [&](int r, int x) {
            const int o = r * TS * 8 + x;
            const unsigned long long two =
                ((unsigned long long)Tw[(o >> 2) + 1] << 32) | Tw[o >> 2];
            return (uint32_t)(two >> (8 * (o & 3)));
        };
        store_tile_bytes(d->labels, d, xs, nx, j0, k0,
                         [&](int r, int x) { return (uint32_t)Tb[r * TS * 8 + x]; }, quad);
        if (d->decisions)
            store_tile_bytes(d->decisions, d, xs, nx, j0, k0, [](int, int) { return 0u; },
                             [](int, int) { return 0u; });
    }
}

// ------------------------------------------------------------------------------------
// Extrapolation of the layer-l cells of one brick, staged in LDS.
// ------------------------------------------------------------------------------------
// Staged cell states (one byte per cell of the 12^3 region).
constexpr uint8_t kStNone = 0;   // carries no data for layer l (outside the box, unmarked,
                                 // or in layer l or above); its staged xi is 0
constexpr uint8_t kStData = 1;   // a datum for layer l: label in [0, l)
constexpr uint8_t kStTarget = 2; // a cell of layer l

// Reciprocal lengths 1/|x'| (in units of the smallest spacing) of the radius-2 offsets:
// entry (|dx| * 3 + |dy|) * 3 + |dz| is 1 / |(dx rho_x, dy rho_y, dz rho_z)| (eq. (weight)
// with the spacings of the axes); d == nullptr or equal spacings: 1 / |d|.
constexpr int kRlen = 27;

__device__ __forceinline__ double rlen_entry(const DevSolid* d, int e) {
    const int ax = e / 9, ay = (e / 3) % 3, az = e % 3;
    if (e == 0) return 0.0;
    if (d == nullptr || !d->aniso) return c_rlen[ax * ax + ay * ay + az * az];
    return 1.0 / norm3((double)ax * d->rho[0], (double)ay * d->rho[1], (double)az * d->rho[2]);
}

// Moments of the eligible data of radius r_s = 2 around staged cell idx.  The staged
// values are xi - A for the brick's anchor A (0 where the cell carries no data), so a
// datum enters as w * v with no selection of the value.  A lane takes whole rows
// (dy, dz); within a row the five data (dx = -2..2) are first summed into row moments
// (sum w, sum w dx, sum w dx^2, sum w v, sum w dx v), which then update the 4 x 4 normal
// matrix and the right-hand sides once per row.  Eq. (weight): w = 2^-(|dx|+|dy|+|dz|),
// times, with the normal, (x_e - x_d).n / |x_e - x_d| where that is positive; the sign
// is decided on (dx gx + dy gy) + dz gz, in that order, without contraction.  The integer
// moments of the positive-weight offsets (for the exact rank test) are summed the same way.
template <int NL, bool NRM, typename T>
__device__ __forceinline__ void gather_lds(const T* __restrict__ sx,
                                           const uint8_t* __restrict__ ss,
                                           const double* __restrict__ s_rlen, int idx,
                                           double g0, double g1, double g2, double rgn, int lq,
                                           Moments<T>& acc) {
    constexpr int S = kBrickSpan, S2 = kBrickSpan * kBrickSpan;
#pragma unroll 1
    for (int row = lq; row < 25; row += NL) {
        const int dy = row % 5 - 2, dz = row / 5 - 2;
        const int rb = idx + dz * S2 + dy * S;
        int st[5];
        T v0[5], v1[5], v2[5];
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int q = rb + u - 2;
            st[u] = ss[q];
            v0[u] = sx[q];
            v1[u] = sx[kBrickCells + q];
            v2[u] = sx[2 * kBrickCells + q];
        }
        const int rowi = abs(dy) * 3 + abs(dz);   // s_rlen entry of (0, dy, dz)
        const double rowbase = ldexp(1.0, -(abs(dy) + abs(dz)));   // 2^-(|dy|+|dz|), exact
        double ry = 0.0, rz = 0.0;
        if (NRM) {
#pragma clang fp contract(off)
            ry = (double)dy * g1;
            rz = (double)dz * g2;
        }
        T s0 = T(0), s1 = T(0), s2 = T(0);
        T t0[3] = {T(0), T(0), T(0)}, t1[3] = {T(0), T(0), T(0)};
        int n = 0, nx = 0, nxx = 0;
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int dx = u - 2;
            bool e = st[u] == kStData;
            double ww = rowbase * (dx == 0 ? 1.0 : (dx == 1 || dx == -1 ? 0.5 : 0.25));
            if (NRM) {
#pragma clang fp contract(off)
                const double dot = ((double)dx * g0 + ry) + rz;
                e = e && (dot < 0.0);
                ww = (-dot * s_rlen[abs(dx) * 9 + rowi] * rgn) * ww;
            }
            const T w = e ? (T)ww : T(0);
            s0 += w;
            t0[0] = fma(w, v0[u], t0[0]);
            t0[1] = fma(w, v1[u], t0[1]);
            t0[2] = fma(w, v2[u], t0[2]);
            if (dx != 0) {   // resolved at compile time (the loop is unrolled)
                const T wx = (T)dx * w;
                s1 += wx;
                s2 = fma((T)dx, wx, s2);
                t1[0] = fma(wx, v0[u], t1[0]);
                t1[1] = fma(wx, v1[u], t1[1]);
                t1[2] = fma(wx, v2[u], t1[2]);
            }
            const int ei = e ? 1 : 0;
            n += ei;
            nx += ei * dx;
            nxx += ei * dx * dx;
        }
        const T fy = (T)dy, fz = (T)dz;
        acc.m[0] += s0;
        acc.m[1] += s1;
        acc.m[2] = fma(fy, s0, acc.m[2]);
        acc.m[3] = fma(fz, s0, acc.m[3]);
        acc.m[4] += s2;
        acc.m[5] = fma(fy, s1, acc.m[5]);
        acc.m[6] = fma(fz, s1, acc.m[6]);
        acc.m[7] = fma(fy * fy, s0, acc.m[7]);
        acc.m[8] = fma(fy * fz, s0, acc.m[8]);
        acc.m[9] = fma(fz * fz, s0, acc.m[9]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc.r[c] += t0[c];
            acc.r[3 + c] += t1[c];
            acc.r[6 + c] = fma(fy, t0[c], acc.r[6 + c]);
            acc.r[9 + c] = fma(fz, t0[c], acc.r[9 + c]);
        }
        acc.g[0] += n + (nxx << 16);
        acc.g[1] += nx + ((dy * nx) << 16);
        acc.g[2] += dy * n + ((dz * nx) << 16);
        acc.g[3] += dz * n + ((dy * dy * n) << 16);
        acc.g[4] += dy * dz * n + ((dz * dz * n) << 16);
    }
}

// The fits of the compacted layer-l cells of a staged brick, NL lanes per cell.  Values
// are relative to the brick's anchor A: xi_e = A + the fitted intercept.
template <int NL, typename T>
__device__ __forceinline__ void fit_cells(const Batch& b, const DevSolid* d,
                                          unsigned long long* st, int l, int ox, int oy, int oz,
                                          int total, unsigned char* lds, const double* s_rlen,
                                          const double* s_anchor) {
    const T* sx = reinterpret_cast<const T*>(lds);
    const uint8_t* ss = reinterpret_cast<const uint8_t*>(lds + kBrickCells * 3 * sizeof(T));
    const uint16_t* cells =
        reinterpret_cast<const uint16_t*>(lds + kBrickCells * (3 * sizeof(T) + 1));
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
    const int64_t nc = d->ncell;
    const double* __restrict__ xi = d->xi;
    const int8_t* __restrict__ labels = d->labels;
    const int grp = threadIdx.x / NL, lq = threadIdx.x % NL;
    const double* rho = d->aniso ? d->rho : nullptr;
    for (int ci = grp; ci < total; ci += 256 / NL) {
        const int idx = cells[ci];
        const int x = idx % kBrickSpan, y = (idx / kBrickSpan) % kBrickSpan,
                  z = idx / (kBrickSpan * kBrickSpan);
        CellCtx cx;
        cx.i = ox + x;
        cx.j = oy + y;
        cx.k = oz + z;
        cx.n0 = n0;
        cx.n1 = n1;
        cx.n2 = n2;
        cx.le = l;
        cx.ncell = nc;
        cx.xi = xi;
        cx.labels = labels;
        const int32_t cell = (cx.k * n1 + cx.j) * n0 + cx.i;
        const bool nrm = l <= b.normal_layers;
        double gn0 = 0.0, gn1 = 0.0, gn2 = 0.0;
        if (nrm) {   // issued first: the only global loads of the cell
            gn0 = d->normals[cell];
            gn1 = d->normals[nc + cell];
            gn2 = d->normals[2 * nc + cell];
        }
        cx.anchor = cell;
        cx.g0 = gn0;
        cx.g1 = gn1;
        cx.g2 = gn2;
        cx.rgn = 0.0;
        cx.rho = rho;
        const bool has_normal = nrm && (gn0 != 0.0 || gn1 != 0.0 || gn2 != 0.0);
        // the physical gradient is g / rho up to a common factor (1 / h)
        if (has_normal)
            cx.rgn = rho ? rlen_scaled(d->irho, gn0, gn1, gn2) : 1.0 / norm3(gn0, gn1, gn2);
        const bool no_normal = nrm && !has_normal;

        // Passes: radii r_s..r_max with eq. (weight), then F1 (normal factor dropped) at
        // r_max, then F2 (kernel-weighted mean) at r_max.
        int code = -1;
        double res[3] = {0.0, 0.0, 0.0};
        const int nfit = b.r_max - b.r_s + 1;
        for (int pass = 0; pass <= nfit + 1; ++pass) {
            const bool f1 = pass == nfit, f2 = pass == nfit + 1;
            if (f1 && !has_normal) continue;
            const int r = (f1 || f2) ? b.r_max : b.r_s + pass;
            const bool un = has_normal && !f1 && !f2;
            Moments<T> acc;
            zero(acc);
            if (r == kBrickHalo) {
                if (un)
                    gather_lds<NL, true, T>(sx, ss, s_rlen, idx, cx.g0, cx.g1, cx.g2, cx.rgn, lq,
                                            acc);
                else
                    gather_lds<NL, false, T>(sx, ss, s_rlen, idx, 0.0, 0.0, 0.0, 0.0, lq, acc);
            } else {
                cx.a0 = s_anchor[0];
                cx.a1 = s_anchor[1];
                cx.a2 = s_anchor[2];
                gather_any<NL, T>(cx, r, un, lq, acc);
            }
            reduce_lanes<NL>(acc);
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
            d->xi[cell] = s_anchor[0] + res[0];
            d->xi[nc + cell] = s_anchor[1] + res[1];
            d->xi[2 * nc + cell] = s_anchor[2] + res[2];
            if (d->decisions) d->decisions[cell] = (int8_t)(code + (no_normal ? kDecNoNormal : 0));
            if (code == kDecF1) atomicAdd(st + ST_F1, 1ull);
            if (code == kDecF2) atomicAdd(st + ST_F2, 1ull);
            if (code == kDecF1 || code == kDecF2 || code > b.r_s) atomicAdd(st + ST_GROWN, 1ull);
        }
    }
}

template <typename T>
__device__ __forceinline__ void extrap_brick(const Batch& b, int s, unsigned long long* st,
                                             int l, int bx, int by, int bz,
                                             unsigned char* lds, int* s_wave,
                                             double* s_anchor, double* s_rlen, int& tab) {
    const DevSolid* d = b.solids + s;
    // the table this brick needs (read before the staging, off the barriers' path)
    const int want = d->aniso ? s : -1;
    T* sx = reinterpret_cast<T*>(lds);
    uint8_t* ss = reinterpret_cast<uint8_t*>(lds + kBrickCells * 3 * sizeof(T));
    uint16_t* cells = reinterpret_cast<uint16_t*>(lds + kBrickCells * (3 * sizeof(T) + 1));
    // re-derived per brick: the staging index math is not kept live across bricks
    const int tid = opaque_lane_value(threadIdx.x);
    const int lane = tid & 63, wid = tid >> 6;
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
    const int64_t nc = d->ncell;
    const double* __restrict__ xi = d->xi;
    const int8_t* __restrict__ labels = d->labels;
    const int ox = kBrick * bx - kBrickHalo, oy = kBrick * by - kBrickHalo,
              oz = kBrick * bz - kBrickHalo;
    // Stage labels and xi of the 12^3 cells.  All loads of the thread are issued before
    // its first LDS store (the stores cannot be moved above them), so the staging costs
    // one round trip.  A cell outside the box loads cell 0 of the box, always there, and
    // is replaced by "no data": no load waits on a branch.
    // The labels are loaded first: the anchor search below needs only them (loads
    // complete in issue order), so it overlaps the xi loads still in flight.
    constexpr int kH = (kBrickCells + 255) / 256;
    int lraw[kH];  // the label loaded (cell 0's outside the box)
    int cidx[kH];  // the cell loaded (0 outside the box)
    unsigned inmask = 0u;   // bit h: cell h of the thread lies in the box
    double v0[kH], v1[kH], v2[kH];
#pragma unroll
    for (int h = 0; h < kH; ++h) {
        const int q = tid + 256 * h;
        const int x = q % kBrickSpan, y = (q / kBrickSpan) % kBrickSpan,
                  z = q / (kBrickSpan * kBrickSpan);
        const int gx = ox + x, gy = oy + y, gz = oz + z;
        const bool in = q < kBrickCells && (unsigned)gx < (unsigned)n0 &&
                        (unsigned)gy < (unsigned)n1 && (unsigned)gz < (unsigned)n2;
        cidx[h] = in ? (gz * n1 + gy) * n0 + gx : 0;
        inmask |= in ? 1u << h : 0u;
        lraw[h] = load_global(labels + cidx[h]);
    }
#pragma unroll
    for (int h = 0; h < kH; ++h) {
        const int c = cidx[h];
        v0[h] = load_global(xi + c);
        v1[h] = load_global(xi + nc + c);
        v2[h] = load_global(xi + 2 * nc + c);
    }
    // nothing that uses a loaded label may be scheduled above the xi loads
    __builtin_amdgcn_sched_barrier(0);
    int lbv[kH];   // the cell's label, -1 outside the box
#pragma unroll
    for (int h = 0; h < kH; ++h) lbv[h] = (inmask >> h) & 1u ? lraw[h] : -1;
    // The brick's anchor A: xi of the first staged cell (in staging order) that carries
    // data for layer l; one exists, since every layer-l cell has a face neighbour in layer
    // l - 1.  Staged values are xi - A: the fit is invariant to the shift, and the
    // offsets are small (the region spans 12 cells), which keeps the moments accurate and
    // lets the reduced-precision form hold them in FP32.
    // (The wave's first such cell: staged cells q = tid + 256 h are in order of h first,
    // so it is the lowest lane of the first slot h whose ballot is not empty.)
    int qf = 0x7fffffff;
#pragma unroll
    for (int h = kH - 1; h >= 0; --h) {
        const unsigned long long m = __ballot(lbv[h] >= 0 && lbv[h] < l);
        if (m) qf = 256 * h + 64 * wid + __builtin_ctzll(m);
    }
    if (lane == 0) s_wave[wid] = qf;
    __syncthreads();
    // the reciprocal-length table of the solid's spacings, when another one is loaded
    // (uniform: the table's owner is the same in every thread)
    if (want != tab) {
        if (tid < kRlen) s_rlen[tid] = rlen_entry(d, tid);
        tab = want;
    }
    const int qa = min(min(s_wave[0], s_wave[1]), min(s_wave[2], s_wave[3]));
    if (qa != 0x7fffffff && (qa & 255) == tid) {
#pragma unroll
        for (int h = 0; h < kH; ++h)
            if (h == (qa >> 8)) {
                s_anchor[0] = v0[h];
                s_anchor[1] = v1[h];
                s_anchor[2] = v2[h];
            }
    }
    if (qa == 0x7fffffff && tid == 0) s_anchor[0] = s_anchor[1] = s_anchor[2] = 0.0;
    __syncthreads();
    const double A0 = s_anchor[0], A1 = s_anchor[1], A2 = s_anchor[2];
#pragma unroll
    for (int h = 0; h < kH; ++h) {
        const int q = tid + 256 * h;
        if (q < kBrickCells) {
            const bool data = lbv[h] >= 0 && lbv[h] < l;
            ss[q] = data ? kStData : (lbv[h] == l ? kStTarget : kStNone);
            sx[q] = data ? (T)(v0[h] - A0) : T(0);
            sx[kBrickCells + q] = data ? (T)(v1[h] - A1) : T(0);
            sx[2 * kBrickCells + q] = data ? (T)(v2[h] - A2) : T(0);
        }
    }
    __syncthreads();
    // the layer-l cells of the brick interior, compacted
    int mine[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = tid + 256 * h;
        const int x = kBrickHalo + q % kBrick, y = kBrickHalo + (q / kBrick) % kBrick,
                  z = kBrickHalo + q / (kBrick * kBrick);
        const int idx = (z * kBrickSpan + y) * kBrickSpan + x;
        mine[h] = ss[idx] == kStTarget ? idx : -1;
    }
    int total = 0;
    {   // by ballots: wave sums, then each cell's place within its wave
        const unsigned long long b0 = __ballot(mine[0] >= 0), b1 = __ballot(mine[1] >= 0);
        const unsigned long long lt = (1ull << lane) - 1ull;
        __syncthreads();   // (s_wave was read for the anchor)
        if (lane == 0) s_wave[wid] = __popcll(b0) + __popcll(b1);
        __syncthreads();
        int wb = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = s_wave[i];
            if (i < wid) wb += t;
            total += t;
        }
        if (mine[0] >= 0) cells[wb + __popcll(b0 & lt)] = (uint16_t)mine[0];
        if (mine[1] >= 0) cells[wb + __popcll(b0) + __popcll(b1 & lt)] = (uint16_t)mine[1];
        __syncthreads();
    }

    // lanes per cell: as many as keep every cell of the brick in one pass of the block
    if (total <= 256 / 16)
        fit_cells<16, T>(b, d, st, l, ox, oy, oz, total, lds, s_rlen, s_anchor);
    else if (total <= 256 / 8)
        fit_cells<8, T>(b, d, st, l, ox, oy, oz, total, lds, s_rlen, s_anchor);
    else
        fit_cells<4, T>(b, d, st, l, ox, oy, oz, total, lds, s_rlen, s_anchor);
    __syncthreads();   // the LDS is reused by the next brick
}

// ------------------------------------------------------------------------------------
// Brick lists: the bucket counts of layers l0..l0+nl-1 form one prefix in LDS
// (s_pref[0..nl*kBuckets]); entry e of the concatenation is found by bisection.  The
// normal kernel walks the bucketed lists this way and copies them into dense per-layer
// lists for the fits.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int list_prefix(const Batch& b, int l0, int nl, int* s_pref,
                                           int* s_wave) {
    const int n = nl * kBuckets;   // <= 1024: four counts per thread
    int v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {   // the four loads first
        const int i = threadIdx.x * 4 + q;
        v[q] = i < n ? b.bcount[(l0 - 1) * kBuckets + i] : 0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = threadIdx.x * 4 + q;
        if (i < n) {
            const int bk = i % kBuckets;
            const int64_t cap = bucket_base(bk + 1, b.n_tiles, b.tile_w) -
                                bucket_base(bk, b.n_tiles, b.tile_w);
            // entries past a bucket's capacity were never written (reported as overflow)
            v[q] = (int)min((int64_t)v[q], cap);
        }
        sum += v[q];
    }
    int excl, total;
    block_scan<4>(sum, excl, total, s_wave);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = threadIdx.x * 4 + q;
        if (i < n) s_pref[i] = excl;
        excl += v[q];
    }
    if (threadIdx.x == 0) s_pref[n] = total;
    __syncthreads();
    return total;
}

// Entry e of the concatenated lists: its layer and list entry.
__device__ __forceinline__ unsigned long long list_entry(const Batch& b, int l0, int nl,
                                                         const int* s_pref, int e, int* layer) {
    int lo = 0, hi = nl * kBuckets - 1;   // last i with s_pref[i] <= e
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pref[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int li = lo / kBuckets, bk = lo % kBuckets;
    *layer = l0 + li;
    return b.blist[(int64_t)(l0 - 1 + li) * b.blist_cap + bucket_base(bk, b.n_tiles, b.tile_w) +
                   (e - s_pref[lo])];
}

// ------------------------------------------------------------------------------------
// Per-solid statistics from the tile counts, then the normals of the listed bricks of
// layers 1..normal_layers.
// ------------------------------------------------------------------------------------
constexpr int kNSpan = kBrick + 2;                        // brick with a halo of 1
constexpr int kNCells = kNSpan * kNSpan * kNSpan;         // 1000

template <bool kSpheres>
__device__ __forceinline__ void normal_brick(const DevSolid* d, unsigned long long* st, int l,
                                             int bx, int by, int bz, double* s_phi,
                                             unsigned char* s_flag, int8_t* s_lab,
                                             uint16_t* s_list, int* s_wave) {
    // re-derived per brick: the index math is not kept live across bricks
    const int tid = opaque_lane_value(threadIdx.x);
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
    const int64_t nc = d->ncell;
    const int ox = kBrick * bx - 1, oy = kBrick * by - 1, oz = kBrick * bz - 1;
    for (int q = tid; q < kNCells; q += 256) s_flag[q] = 0;
    const int8_t* __restrict__ labels = d->labels;
    int8_t lv[2];   // both label loads issued before the LDS stores
    bool inb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = tid + 256 * h;
        const int x = q % kBrick, y = (q / kBrick) % kBrick, z = q / (kBrick * kBrick);
        const int gx = ox + 1 + x, gy = oy + 1 + y, gz = oz + 1 + z;
        inb[h] = gx < n0 && gy < n1 && gz < n2;
        lv[h] = load_global(labels + (inb[h] ? ((int64_t)gz * n1 + gy) * n0 + gx : 0));
    }
    s_lab[tid] = inb[0] ? lv[0] : (int8_t)-1;
    s_lab[tid + 256] = inb[1] ? lv[1] : (int8_t)-1;
    __syncthreads();
    // a cell of layer l needs phi0 at itself and at its six face neighbours
    for (int q = tid; q < kBrick * kBrick * kBrick; q += 256) {
        if (s_lab[q] != l) continue;
        const int x = q % kBrick, y = (q / kBrick) % kBrick, z = q / (kBrick * kBrick);
        const int r = ((z + 1) * kNSpan + (y + 1)) * kNSpan + (x + 1);
        s_flag[r] = 1;
        s_flag[r - 1] = 1;
        s_flag[r + 1] = 1;
        s_flag[r - kNSpan] = 1;
        s_flag[r + kNSpan] = 1;
        s_flag[r - kNSpan * kNSpan] = 1;
        s_flag[r + kNSpan * kNSpan] = 1;
    }
    __syncthreads();
    // compact the needed cells: region cell q = tid + 256 h, by ballots (the list's order
    // does not matter)
    int total = 0;
    {
        const int lane = tid & 63, wid = tid >> 6;
        const unsigned long long lt = (1ull << lane) - 1ull;
        unsigned long long bal[4];
        int wsum = 0;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int q = tid + 256 * h;
            bal[h] = __ballot(q < kNCells && s_flag[q]);
            wsum += __popcll(bal[h]);
        }
        if (lane == 0) s_wave[wid] = wsum;
        __syncthreads();
        int pos = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = s_wave[i];
            if (i < wid) pos += t;
            total += t;
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int q = tid + 256 * h;
            if ((bal[h] >> lane) & 1ull) s_list[pos + __popcll(bal[h] & lt)] = (uint16_t)q;
            pos += __popcll(bal[h]);
        }
        __syncthreads();
    }
    // phi0 of each needed cell once (defined: inside the box with a finite xi)
    const ShapeR sh = load_shape(d);
    const double* __restrict__ f = d->xi_normal;
    for (int i = tid; i < total; i += 256) {
        const int r = s_list[i];
        const int x = r % kNSpan, y = (r / kNSpan) % kNSpan, z = r / (kNSpan * kNSpan);
        const int gx = ox + x, gy = oy + y, gz = oz + z;
        const bool in = (unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1 &&
                        (unsigned)gz < (unsigned)n2;
        const int64_t c = in ? ((int64_t)gz * n1 + gy) * n0 + gx : 0;
        const double x0 = load_global(f + c), x1 = load_global(f + nc + c),
                     x2 = load_global(f + 2 * nc + c);
        const bool def = in && finite3(x0, x1, x2);
        double ph = 0.0;
        if (def) {
            if constexpr (kSpheres)
                ph = phi0_sphere(sh, x0, x1, x2);
            else
                ph = phi0(sh, x0, x1, x2);
        }
        s_phi[r] = ph;
        s_flag[r] = def ? 3 : 1;
    }
    __syncthreads();
    // central differences where both neighbours are defined, else one-sided with the cell
    // itself (forward first), else 0
    int nzero = 0;
    for (int q = tid; q < kBrick * kBrick * kBrick; q += 256) {
        if (s_lab[q] != l) continue;
        const int x = q % kBrick, y = (q / kBrick) % kBrick, z = q / (kBrick * kBrick);
        const int r = ((z + 1) * kNSpan + (y + 1)) * kNSpan + (x + 1);
        const int step[3] = {1, kNSpan, kNSpan * kNSpan};
        const bool d0 = s_flag[r] == 3;
        double g[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int rp = r + step[a], rm = r - step[a];
            const bool dp = s_flag[rp] == 3, dm = s_flag[rm] == 3;
            double ga;
            if (dp && dm) ga = 0.5 * (s_phi[rp] - s_phi[rm]);
            else if (dp && d0) ga = s_phi[rp] - s_phi[r];
            else if (dm && d0) ga = s_phi[r] - s_phi[rm];
            else ga = 0.0;
            g[a] = ga;
        }
        const int64_t cell = ((int64_t)(oz + 1 + z) * n1 + (oy + 1 + y)) * n0 + (ox + 1 + x);
        d->normals[cell] = g[0];
        d->normals[nc + cell] = g[1];
        d->normals[2 * nc + cell] = g[2];
        nzero += (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0);
    }
    if (nzero) atomicAdd(st + ST_NONORMAL, (unsigned long long)nzero);   // rare
}

// Per-solid interior and band counts, the sums of the solids' tile counts, into the
// statistics (blocks b, b + gridDim.x, ... take solids b, ...).
__device__ __forceinline__ void solid_counts(const Batch& b, unsigned long long* s_acc) {
    const int tid = threadIdx.x;
    for (int s = blockIdx.x; s < b.n_solids; s += gridDim.x) {
        const DevSolid* d = b.solids + s;
        if (tid < kLT) s_acc[tid] = 0ull;
        __syncthreads();
        // (a count is at most the box's cells, below 2^31: 32-bit sums)
        int acc[kLT];
#pragma unroll
        for (int l = 0; l < kLT; ++l) acc[l] = 0;
        const int L = d->L;
        for (int t = d->tile_base + tid; t < d->tile_base + d->n_tiles; t += 256) {
            // every count of the tile loaded at once (entries past L hold no count of
            // this call and are dropped)
            int v[kLT];
#pragma unroll
            for (int l = 0; l < kLT; ++l) v[l] = b.tile_cnt[(int64_t)t * kLT + l];
#pragma unroll
            for (int l = 0; l < kLT; ++l) acc[l] += l <= L ? v[l] : 0;
        }
        // wave sums first (DPP row sums and four lane reads): one LDS atomic per wave and
        // count
#pragma unroll
        for (int l = 0; l < kLT; ++l) {
            if (l <= L) {   // uniform
                const int v = wave_sum(acc[l]);
                if ((tid & 63) == 0 && v) atomicAdd(&s_acc[l], (unsigned long long)(unsigned)v);
            }
        }
        __syncthreads();
        if (tid < kLT) b.stats[(int64_t)s * kStatWords + tid] = s_acc[tid];
        __syncthreads();
    }
}

// Four waves per SIMD (at most 128 registers, none spilled): the blocks go through their
// bricks' bisections one at a time, so resident waves hide the divide chains.  A call
// whose solids are all spheres takes the sphere-only form (kSpheres), which holds no
// bisection and keeps more blocks resident.
template <bool kSpheres>
__global__ __launch_bounds__(256, kSpheres ? 8 : 4) void k_normal(Batch b) {
    __shared__ int s_wave[4];
    __shared__ int s_pref[kMaxLayers * kBuckets + 1];
    __shared__ unsigned long long s_acc[kLT];
    __shared__ double s_phi[kNCells];
    __shared__ unsigned char s_flag[kNCells];
    __shared__ int8_t s_lab[kBrick * kBrick * kBrick];
    __shared__ uint16_t s_list[kNCells];
    const int tid = threadIdx.x;
    solid_counts(b, s_acc);
    // Dense per-layer brick lists for the fits: entry e of the bucketed lists of layers
    // 1..Lmax goes to its rank within its layer (bucket order), and each layer's count to
    // dcount.  The prefix over all layers also serves the normals' layers 1..nl.
    const int tot = list_prefix(b, 1, b.Lmax, s_pref, s_wave);
    if (blockIdx.x == 0 && tid < b.Lmax)
        b.dcount[tid] = s_pref[(tid + 1) * kBuckets] - s_pref[tid * kBuckets];
    for (int e = blockIdx.x * 256 + tid; e < tot; e += gridDim.x * 256) {
        int layer = 1;
        const unsigned long long pk = list_entry(b, 1, b.Lmax, s_pref, e, &layer);
        const int64_t i = e - s_pref[(layer - 1) * kBuckets];
        if (i < b.dlist_cap) b.dlist[(int64_t)(layer - 1) * b.dlist_cap + i] = pk;
    }
    const int nl = b.normal_layers;
    if (nl <= 0) return;
    const int total = s_pref[nl * kBuckets];
    const XcdRange rg = xcd_range(total);
    for (int e = rg.begin; e < rg.end; e += rg.stride) {
        int l = 0;
        const unsigned long long pk = list_entry(b, 1, nl, s_pref, e, &l);
        const int s = uniform_int((int)(pk >> 32));
        const int bx = uniform_int((int)(pk & 1023ull));
        const int by = uniform_int((int)((pk >> 10) & 1023ull));
        const int bz = uniform_int((int)((pk >> 20) & 1023ull));
        l = uniform_int(l);
        unsigned long long* st = b.stats + (int64_t)s * kStatWords;
        if (st[ST_FLAGS] & FLAG_TRUNCATED) continue;   // uniform: no fit follows
        normal_brick<kSpheres>(b.solids + s, st, l, bx, by, bz, s_phi, s_flag, s_lab, s_list,
                               s_wave);
        __syncthreads();   // the LDS is reused by the next brick
    }
}

// One launch per layer over the layer's dense brick list (built by the normal kernel):
// the blocks of each XCD stride over a contiguous range of it, so neighbouring bricks,
// whose halos overlap, share one L2.
template <typename T>
__global__ __launch_bounds__(256, 3) void k_extrap(Batch b, int l) {
    HIP_DYNAMIC_SHARED(double, lds_d)
    unsigned char* lds = reinterpret_cast<unsigned char*>(lds_d);
    __shared__ int s_wave[4];
    __shared__ double s_anchor[3];
    __shared__ double s_rlen[kRlen];
    if (threadIdx.x < kRlen) s_rlen[threadIdx.x] = rlen_entry(nullptr, threadIdx.x);
    int tab = -1;   // the loaded table: equal spacings
    const unsigned long long* dl = b.dlist + (int64_t)(l - 1) * b.dlist_cap;
    const int count = uniform_int((int)min((int64_t)b.dcount[l - 1], b.dlist_cap));
    __syncthreads();   // s_rlen
    const XcdRange rg = xcd_range(count);
    for (int e = rg.begin; e < rg.end; e += rg.stride) {
        const unsigned long long pk = dl[e];
        const int s = uniform_int((int)(pk >> 32));
        const int bx = uniform_int((int)(pk & 1023ull));
        const int by = uniform_int((int)((pk >> 10) & 1023ull));
        const int bz = uniform_int((int)((pk >> 20) & 1023ull));
        unsigned long long* st = b.stats + (int64_t)s * kStatWords;
        if (st[ST_FLAGS] & FLAG_TRUNCATED) continue;   // uniform: whole block skips
        extrap_brick<T>(b, s, st, l, bx, by, bz, lds, s_wave, s_anchor, s_rlen, tab);
    }
}


// ------------------------------------------------------------------------------------
// Persistent band launch: the normals and the fits of every layer of the whole batch in
// ONE launch, over the compacted brick lists.  Work items are bricks: phase 0 the bricks
// of layers 1..normal_layers (normals), phase l the bricks of layer l (fits).  Each phase
// is split into kQueues contiguous slices, one queue each, in proportion to the blocks of
// queue x (blocks b with b % kQueues == x): neighbouring bricks, whose halos overlap, are
// then mostly fitted on one XCD (the hardware deals blocks to the XCDs round-robin).  A
// block takes items of its current phase from its own queue, then from any queue with
// items left, and moves to the next phase only once every queue of its phase is
// exhausted.  An item of phase p > 0 waits until every item of phase p - 1 is complete
// (layers in ascending order, "Extrapolation of xi"; the normals are taken from the field
// before any fit writes).  A block publishes its finished items of a phase (one release,
// one count) when it leaves the phase, before it can wait; it acquires once per phase it
// enters, and polls without ordering: an ordered poll would invalidate the XCD's L2 on
// every read.  Since no block reaches phase p before all items of phase p - 1 were
// handed out, each to a block that is running, the lowest unfinished phase always has
// its items in blocks that do not wait: no deadlock, whatever the residency.  Every wait
// is bounded: past the bound the call's error flag is set, the item is skipped (still
// counted), and every wave reaches the end.
// ------------------------------------------------------------------------------------
constexpr int kQueues = kXcds;
constexpr int kBandSpin = 1 << 20;   // polls of a bounded wait (each an acquire load and a
                                     // short sleep: about a second in all)

// Shared memory of the band kernel, carved from its dynamic LDS (no static LDS: the
// block's whole state lies in its own allocation).
struct BandLds {
    unsigned char* work;   // a brick's fit staging, or a brick's normal scratch
    double* s_phi;
    unsigned char* s_flag;
    int8_t* s_lab;
    uint16_t* s_list;
    int* s_pref;           // [kMaxLayers * kBuckets + 1]
    int* s_wave;           // [4]
    int* s_ctl;            // [4]: ticket, wait result
    double* s_anchor;      // [3]
    double* s_rlen;        // [kRlen]
    unsigned long long* s_acc;  // [kLT]
};

__host__ __device__ constexpr size_t band_small_bytes() {
    return sizeof(int) * (kMaxLayers * kBuckets + 1 + 4 + 4) + sizeof(double) * (3 + kRlen) +
           sizeof(unsigned long long) * kLT + 64;
}

__device__ __forceinline__ BandLds band_lds(unsigned char* lds, size_t work_bytes) {
    BandLds L;
    L.work = lds;
    L.s_phi = reinterpret_cast<double*>(lds);
    L.s_flag = lds + sizeof(double) * kNCells;
    L.s_lab = reinterpret_cast<int8_t*>(L.s_flag + kNCells);
    L.s_list = reinterpret_cast<uint16_t*>(lds + sizeof(double) * kNCells + kNCells +
                                           kBrick * kBrick * kBrick);
    unsigned char* sm = lds + ((work_bytes + 15) & ~size_t(15));
    L.s_anchor = reinterpret_cast<double*>(sm);
    L.s_rlen = L.s_anchor + 3;
    L.s_acc = reinterpret_cast<unsigned long long*>(L.s_rlen + kRlen);
    L.s_pref = reinterpret_cast<int*>(L.s_acc + kLT);
    L.s_wave = L.s_pref + kMaxLayers * kBuckets + 1;
    L.s_ctl = L.s_wave + 4;
    return L;
}

// Items of phase p (0: bricks of layers 1..nl; p >= 1: bricks of layer p).
__device__ __forceinline__ int phase_items(const int* s_pref, int p, int nl) {
    return p == 0 ? s_pref[nl * kBuckets] : s_pref[p * kBuckets] - s_pref[(p - 1) * kBuckets];
}

// Slice [lo, hi) of a phase's n items held by queue x of nq, over G blocks.
__device__ __forceinline__ void queue_slice(int n, int G, int nq, int x, int* lo, int* hi) {
    int before = 0;   // blocks of the queues before x
    for (int y = 0; y < x; ++y) before += (G - y + nq - 1) / nq;
    const int mine = (G - x + nq - 1) / nq;
    *lo = (int)((int64_t)n * before / G);
    *hi = (int)((int64_t)n * (before + mine) / G);
}

// Wave 0 of a block: the next item of the block's phase *ph (advanced past exhausted
// phases); returns its index within the phase, or -1 once every phase is exhausted.
__device__ int band_take(BandCtl* ctl, const int* s_pref, int nl, int Lmax, int q, int nq,
                         int* ph) {
    const int lane = threadIdx.x;
    const int G = gridDim.x;
    for (; *ph <= Lmax; ++*ph) {
        const int p = *ph;
        const int n = phase_items(s_pref, p, nl);
        int lo, hi;
        queue_slice(n, G, nq, q, &lo, &hi);
        int t = 0;
        if (lane == 0) t = atomicAdd(&ctl->taken[p][q], 1);
        t = __shfl(t, 0);
        if (t < hi - lo) return lo + t;
        // the other queues: lane i < nq - 1 looks at queue (q + 1 + i) % nq
        for (;;) {
            const int x = (q + 1 + lane) % nq;
            int xlo = 0, xhi = 0, left = 0;
            if (lane < nq - 1) {
                queue_slice(n, G, nq, x, &xlo, &xhi);
                left = __hip_atomic_load(&ctl->taken[p][x], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < xhi - xlo;
            }
            const unsigned long long m = __ballot(left);
            if (m == 0ull) break;   // phase exhausted
            const int src = __ffsll((long long)m) - 1;
            int u = 0;
            if (lane == src) u = atomicAdd(&ctl->taken[p][x], 1);
            u = __shfl(u, src);
            const int ulo = __shfl(xlo, src), uhi = __shfl(xhi, src);
            if (u < uhi - ulo) return ulo + u;
        }
    }
    return -1;
}

template <typename T>
__global__ __launch_bounds__(256, 3) void k_band(Batch b, int work_bytes) {
    HIP_DYNAMIC_SHARED(double, lds_d)
    const BandLds L = band_lds(reinterpret_cast<unsigned char*>(lds_d), (size_t)work_bytes);
    BandCtl* ctl = b.band;
    const int tid = threadIdx.x;
    if (tid < kRlen) L.s_rlen[tid] = rlen_entry(nullptr, tid);
    int tab = -1;   // the loaded reciprocal-length table: equal spacings
    solid_counts(b, L.s_acc);
    list_prefix(b, 1, b.Lmax, L.s_pref, L.s_wave);   // (ends with a barrier)
    const int nl = b.normal_layers;
    const int nq = gridDim.x < kQueues ? (int)gridDim.x : kQueues;
    const int q = blockIdx.x % nq;
    int ph = 0, err = 0;
    int ready = 0;              // phases before this one are complete and acquired
    int pend = 0, pend_ph = 0;  // items of phase pend_ph done here and not yet published
    for (;;) {
        if (tid < 64) {
            int p = ph;
            const int it = band_take(ctl, L.s_pref, nl, b.Lmax, q, nq, &p);
            if (tid == 0) {
                L.s_ctl[0] = it;
                L.s_ctl[2] = p;
            }
        }
        __syncthreads();
        const int item = L.s_ctl[0];
        const int p = L.s_ctl[2];
        __syncthreads();   // (s_ctl is rewritten by the next take)
        ph = p;
        // publish this block's finished items of an earlier phase before anything waits:
        // every thread's stores (one release), then their count
        if (pend > 0 && (item < 0 || p != pend_ph)) {
            __threadfence();
            __syncthreads();
            if (tid == 0) atomicAdd(&ctl->done[pend_ph], pend);
            pend = 0;
        }
        if (item < 0) break;   // every phase is exhausted
        bool run = !err;
        if (p > ready) {
            // wait until every item of phase p - 1 is complete (polled without ordering,
            // then one acquire for the whole block)
            if (tid == 0) {
                const int need = phase_items(L.s_pref, p - 1, nl);
                int ok = 1, spins = 0;
                while (__hip_atomic_load(&ctl->done[p - 1], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (++spins > kBandSpin ||
                        __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        atomicOr(&ctl->err, 1);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                L.s_ctl[1] = ok;
            }
            __syncthreads();
            const int ok = L.s_ctl[1];
            run = run && ok;
            err = !ok || err;
            // every thread: its later loads see what the finished items stored
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (ok) ready = p;
        }
        if (run) {
            const int e = p == 0 ? item : L.s_pref[(p - 1) * kBuckets] + item;
            int layer = 1;
            const unsigned long long pk = list_entry(b, 1, b.Lmax, L.s_pref, e, &layer);
            const int s = uniform_int((int)(pk >> 32));
            const int bx = uniform_int((int)(pk & 1023ull));
            const int by = uniform_int((int)((pk >> 10) & 1023ull));
            const int bz = uniform_int((int)((pk >> 20) & 1023ull));
            layer = uniform_int(layer);
            unsigned long long* st = b.stats + (int64_t)s * kStatWords;
            if (!(st[ST_FLAGS] & FLAG_TRUNCATED)) {   // uniform: no fit follows a truncation
                if (p == 0)
                    normal_brick<false>(b.solids + s, st, layer, bx, by, bz, L.s_phi, L.s_flag, L.s_lab,
                                 L.s_list, L.s_wave);
                else
                    extrap_brick<T>(b, s, st, p, bx, by, bz, L.work, L.s_wave, L.s_anchor,
                                    L.s_rlen, tab);
            }
        }
        ++pend;   // (a skipped item counts too)
        pend_ph = p;
        __syncthreads();   // the item's LDS is free for the next one
    }
    if (err && tid == 0)
        for (int s = 0; s < b.n_solids; ++s)
            atomicOr(b.stats + (int64_t)s * kStatWords + ST_FLAGS, FLAG_TIMEOUT);
}

}  // namespace

// ------------------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------------------
hipError_t launch_classify(const Batch& b, hipStream_t st) {
    const int grid = b.n_chunks < 8192 ? b.n_chunks : 8192;
    hipLaunchKernelGGL(k_classify, dim3(grid), dim3(256), 0, st, b);
    return hipGetLastError();
}

size_t label_lds_bytes(int Lmax, int tile_w, int Wmax) {
    const int RJ = kTileJ + 2 * Lmax, RK = kTileK + 2 * Lmax;
    const int RW = tile_w + 2 < Wmax ? tile_w + 2 : Wmax;
    const size_t region = sizeof(unsigned long long) * 2 * (size_t)(RW | 1) * RJ * RK;
    const size_t rows = (size_t)256 * 8 * (8 * tile_w + 1);   // transposed labels of a tile
    return region > rows ? region : rows;
}

hipError_t launch_label(const Batch& b, size_t lds, hipStream_t st) {
    if (b.tile_w == 1)
        hipLaunchKernelGGL(k_label<1>, dim3(b.n_tiles), dim3(kLabelThreads), lds, st, b);
    else if (b.tile_w == 2)
        hipLaunchKernelGGL(k_label<2>, dim3(b.n_tiles), dim3(kLabelThreads), lds, st, b);
    else if (b.tile_w == 4)
        hipLaunchKernelGGL(k_label<4>, dim3(b.n_tiles), dim3(kLabelThreads), lds, st, b);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int normal_blocks_per_cu(bool spheres) {
    static const int n[2] = {[] {
                                 int v = 0;
                                 if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                         &v, k_normal<false>, 256, 0) != hipSuccess || v < 1)
                                     v = 4;
                                 return v;
                             }(),
                             [] {
                                 int v = 0;
                                 if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                         &v, k_normal<true>, 256, 0) != hipSuccess || v < 1)
                                     v = 4;
                                 return v;
                             }()};
    return n[spheres ? 1 : 0];
}

hipError_t launch_normal(const Batch& b, int blocks, hipStream_t st) {
    if (b.spheres)
        hipLaunchKernelGGL(k_normal<true>, dim3(blocks), dim3(256), 0, st, b);
    else
        hipLaunchKernelGGL(k_normal<false>, dim3(blocks), dim3(256), 0, st, b);
    return hipGetLastError();
}

size_t band_lds_bytes(int precision) {
    const size_t normal = sizeof(double) * kNCells + kNCells + kBrick * kBrick * kBrick +
                          sizeof(uint16_t) * kNCells;
    const size_t fit = brick_lds_bytes(precision);
    const size_t work = fit > normal ? fit : normal;
    return ((work + 15) & ~size_t(15)) + band_small_bytes();
}

// Blocks per CU of the persistent launch: one, when one fits.  Each block releases (an L2
// write-back of its XCD) when it leaves a phase and acquires (an L2 invalidation) when it
// enters one; with more blocks per CU these operations thrash the L2 more than the added
// residency hides latency (one block per CU measured twice as fast as three).
int band_blocks_per_cu(int precision) {
    static const int n[2] = {
        [] {
            int v = 0;
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_band<double>, 256,
                                                                band_lds_bytes(0)) == hipSuccess &&
                           v >= 1
                       ? 1
                       : 0;
        }(),
        [] {
            int v = 0;
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_band<float>, 256,
                                                                band_lds_bytes(1)) == hipSuccess &&
                           v >= 1
                       ? 1
                       : 0;
        }()};
    return n[precision == 1 ? 1 : 0];
}

hipError_t launch_band(const Batch& b, int precision, int blocks, hipStream_t st) {
    const size_t lds = band_lds_bytes(precision);
    const int work = (int)(lds - band_small_bytes());
    if (precision == 1)
        hipLaunchKernelGGL(k_band<float>, dim3(blocks), dim3(256), lds, st, b, work);
    else
        hipLaunchKernelGGL(k_band<double>, dim3(blocks), dim3(256), lds, st, b, work);
    return hipGetLastError();
}

hipError_t launch_extrap(const Batch& b, int layer, int precision, int blocks,
                         hipStream_t st) {
    if (precision == 1)
        hipLaunchKernelGGL(k_extrap<float>, dim3(blocks), dim3(256), brick_lds_bytes(1), st, b,
                           layer);
    else
        hipLaunchKernelGGL(k_extrap<double>, dim3(blocks), dim3(256), brick_lds_bytes(0), st, b,
                           layer);
    return hipGetLastError();
}

}  // namespace rmx
