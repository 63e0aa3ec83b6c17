// Phase bodies shared by the per-solid launch chain and the fused persistent kernel:
// classification of a run of 64-cell row segments, and the labelling of one tile.
#pragma once
#include "rmx_device.h"

namespace rmx {
namespace dev {

// ------------------------------------------------------------------------------------
// Classification of mask words [wb, we) of solid d by the 4 waves of the block: each wave
// streams 16 consecutive 64-cell row segments, 8 at a time (24 loads of 512 contiguous
// bytes in flight), ballot-packs the interior predicate and writes one mask word per
// segment.  Returns, per thread, whether it saw an interior cell closer than L to a box
// face that is no grid wall (the band would be truncated).
// ------------------------------------------------------------------------------------
constexpr int kSeg = 8;

__device__ __forceinline__ bool classify_words(const DevSolid* dp, int wb, int we) {
    const int lane = threadIdx.x & 63;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int n0 = dp->n0, n1 = dp->n1, n2 = dp->n2, W = dp->W, L = dp->L;
    const int64_t ncell = dp->ncell;
    const double* __restrict__ xi = dp->xi;
    unsigned long long* __restrict__ mask = dp->mask;
    const bool wl0 = dp->wall_lo[0], wh0 = dp->wall_hi[0];
    const bool wl1 = dp->wall_lo[1], wh1 = dp->wall_hi[1];
    const bool wl2 = dp->wall_lo[2], wh2 = dp->wall_hi[2];
    const ShapeR sh = load_shape(dp);
    const int first = wb + wave * (kChunkWords / 4);
    bool trunc = false;
#pragma unroll 1
    for (int it = 0; it < kChunkWords / 4; it += kSeg) {
        const int w0 = first + it;
        if (w0 >= we) break;
        int row = w0 / W, wx = w0 - row * W;
        double v0[kSeg], v1[kSeg], v2[kSeg];
        int rows[kSeg], xs[kSeg];
#pragma unroll
        for (int u = 0; u < kSeg; ++u) {
            const int x = wx * 64 + lane;
            rows[u] = row;
            xs[u] = x;
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
        for (int u = 0; u < kSeg; ++u) {
            const bool in = interior(sh, v0[u], v1[u], v2[u]);
            const unsigned long long m = __ballot(in);
            if (lane == 0 && w0 + u < we) mask[w0 + u] = m;
            if (m) {
                const int yy = rows[u] % n1, zz = rows[u] / n1, xx = xs[u];
                trunc |= in && ((!wl0 && xx < L) || (!wh0 && n0 - 1 - xx < L) ||
                                (!wl1 && yy < L) || (!wh1 && n1 - 1 - yy < L) ||
                                (!wl2 && zz < L) || (!wh2 && n2 - 1 - zz < L));
            }
        }
    }
    return trunc;
}

// ------------------------------------------------------------------------------------
// Labels of one tile of 16 (y) x 16 (z) rows x tile_w 64-cell words (x); thread (tj, tk)
// owns one row of the tile.  The region in LDS carries a halo of L rows in y and z and
// one word on each side in x where the box continues (L <= 16 < 64), so after L dilations
// through face neighbours (64-bit shifts and ORs) the tile is exact.  The first dilation
// that reaches a cell is its layer.  Per tile it records the interior count and the
// cells of each layer.  The chain form lists the band cells, grouped by layer, in the
// tile's slot range; the fused form computes the normals of the cells of layers
// <= normal_layers and lists the 8^3 bricks that hold cells of each layer.
// ------------------------------------------------------------------------------------
constexpr int kMaxTileW = 4;
constexpr int kRowsPerThread = 9;   // ceil((16 + 2 * 16)^2 / 256)
constexpr int kBrickFlagsPerLayer = 4 * 8;   // fused tiles are one word wide

template <bool FUSED, int MAXTW>
__device__ __forceinline__ void label_tile(const Batch& b, const Fused* f, int t, int s,
                                           const DevSolid* d, unsigned char* ldsraw,
                                           int* s_wave, unsigned char* s_bflag) {
    unsigned long long* lds = reinterpret_cast<unsigned long long*>(ldsraw);
    const int tid = threadIdx.x;
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

    if (FUSED) {
        for (int q = tid; q < kMaxLayers * kBrickFlagsPerLayer; q += 256) s_bflag[q] = 0;
    }
    // Region rows owned by this thread, with their position and box membership.
    // packed per owned row: rj | rk << 8 | in-box << 16 (RJ, RK <= 48)
    int rinfo[kRowsPerThread];
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
        const int rr = tid + 256 * q;
        const int rj = rr % RJ, rk = rr / RJ;
        const int jj = j0 - H + rj, kk = k0 - H + rk;
        const bool ok = rr < R && jj >= 0 && jj < n1 && kk >= 0 && kk < n2;
        rinfo[q] = rj | (rk << 8) | (ok ? 1 << 16 : 0);
        if (rr < R) {
            for (int w = 0; w < RW; ++w)
                A[rr * RW + w] = ok ? mask[((int64_t)kk * n1 + jj) * W + xr0 + w] : 0ull;
        }
    }
    __syncthreads();

    const int tj = tid % kTileJ, tk = tid / kTileJ;
    const int jrow = j0 + tj, krow = k0 + tk;
    const bool row_ok = jrow < n1 && krow < n2;
    const int my = ((tk + H) * RJ + (tj + H)) * RW + (wx0 - xr0);
    unsigned long long prev[MAXTW], p0[MAXTW], p1[MAXTW], p2[MAXTW], p3[MAXTW], p4[MAXTW];
    int cnt0 = 0;
#pragma unroll
    for (int w = 0; w < MAXTW; ++w) {
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
    ShapeR sh;
    if (FUSED) sh = load_shape(d);

    for (int l = 1; l <= L; ++l) {
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
            const int rr = tid + 256 * q;
            if (rr < R) {
                const int rj = rinfo[q] & 255, rk = (rinfo[q] >> 8) & 255;
                const bool rok = (rinfo[q] >> 16) & 1;
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
                    const unsigned long long vm =
                        !rok ? 0ull : (xr0 + w == W - 1 ? tail : ~0ull);
                    B[idx] = v & vm;
                }
            }
        }
        __syncthreads();
        unsigned long long* tmp = A;
        A = B;
        B = tmp;
        unsigned long long nw[MAXTW];
        int cnt = 0;
#pragma unroll
        for (int w = 0; w < MAXTW; ++w) {
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
        if (!FUSED) {
            int64_t pos = tile_slot + lstart + excl;
#pragma unroll
            for (int w = 0; w < MAXTW; ++w) {
                unsigned long long m = nw[w];
                while (m) {
                    const int bit = __ffsll((long long)m) - 1;
                    m &= m - 1ull;
                    b.slots[pos++] = rowbase + w * 64 + bit;
                }
            }
        } else {
            const int bq = (l - 1) * kBrickFlagsPerLayer + ((tk >> 3) * 2 + (tj >> 3)) * 8;
#pragma unroll
            for (int g = 0; g < 8; ++g)
                if ((nw[0] >> (8 * g)) & 255ull) s_bflag[bq + g] = 1;
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
    if (FUSED && row_ok) {
        // Normals of this row's cells of layers 1..normal_layers, from the field before
        // any write (no fit of these slabs has started).
        const int64_t nc = d->ncell;
        const int nl = min(b.normal_layers, L);
        int nzero = 0;
#pragma unroll
        for (int w = 0; w < MAXTW; ++w) {
            for (int l = 1; l <= nl; ++l) {
                unsigned long long m = prev[w];
                m &= (l & 1) ? p0[w] : ~p0[w];
                m &= (l & 2) ? p1[w] : ~p1[w];
                m &= (l & 4) ? p2[w] : ~p2[w];
                m &= (l & 8) ? p3[w] : ~p3[w];
                m &= (l & 16) ? p4[w] : ~p4[w];
                while (m) {
                    const int bit = __ffsll((long long)m) - 1;
                    m &= m - 1ull;
                    const int x = wx0 * 64 + w * 64 + bit;
                    const int32_t cell = rowbase + w * 64 + bit;
                    double g[3];
                    normal_at(sh, d->xi_normal, nc, n0, n1, n2, cell, x, jrow, krow, g);
                    d->normals[cell] = g[0];
                    d->normals[nc + cell] = g[1];
                    d->normals[2 * nc + cell] = g[2];
                    nzero += (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0);
                }
            }
        }
        if (nzero) atomicAdd(f->ctr + d->ctr + 3, nzero);
    }
    if (FUSED) {
        __syncthreads();
        for (int q = tid; q < L * kBrickFlagsPerLayer; q += 256) {
            if (!s_bflag[q]) continue;
            const int l = q / kBrickFlagsPerLayer + 1, r = q % kBrickFlagsPerLayer;
            const int yz = r / 8, bxl = r % 8;
            const int bx = wx0 * 8 + bxl, by = 2 * tyi + (yz & 1), bz = 2 * tzi + (yz >> 1);
            int* cntp = f->ctr + d->ctr + kCtrSolid + (2 + L + (l - 1)) * d->n_slabs + tzi;
            const int pos = atomicAdd(cntp, 1);
            f->lists[d->list + ((int64_t)(l - 1) * d->n_slabs + tzi) * d->bcap + pos] =
                bx | (by << 10) | (bz << 20);
        }
    }

    if (row_ok) {
        int8_t* lab0 = d->labels + ((int64_t)krow * n1 + jrow) * n0 + wx0 * 64;
        int8_t* dec0 = d->decisions ? d->decisions + ((int64_t)krow * n1 + jrow) * n0 + wx0 * 64
                                    : nullptr;
#pragma unroll
        for (int w = 0; w < MAXTW; ++w) {
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
    __syncthreads();   // the LDS region is reused by the block's next item
}

}  // namespace dev
}  // namespace rmx
