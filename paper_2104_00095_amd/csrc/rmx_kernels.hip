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
#include "rmx_device.h"
#include "rmx_fused_common.h"

namespace rmx {
namespace {
using namespace dev;

// ------------------------------------------------------------------------------------
// Classification: a block owns a chunk of kChunkWords mask words of one solid.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_classify(Batch b) {
    for (int chunk = blockIdx.x; chunk < b.n_chunks; chunk += gridDim.x) {
        const int s = uniform_int(find_solid_by_chunk(b.solids, b.n_solids, chunk));
        const DevSolid* dp = b.solids + s;
        const int nwords = dp->n1 * dp->n2 * dp->W;
        const int first = (chunk - dp->chunk_base) * kChunkWords;
        const bool trunc = classify_words(dp, first, min(first + kChunkWords, nwords));
        const int any = __syncthreads_or(trunc);
        if (threadIdx.x == 0) b.chunk_flag[chunk] = any ? 1 : 0;
    }
}

// ------------------------------------------------------------------------------------
// Labels: one workgroup per tile.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_label(Batch b) {
    HIP_DYNAMIC_SHARED(double, lds_d)
    unsigned char* lds = reinterpret_cast<unsigned char*>(lds_d);
    __shared__ int s_wave[4];
    const int t = blockIdx.x;
    const int s = uniform_int(b.tile_solid[t]);
    label_tile<false, kMaxTileW>(b, nullptr, t, s, b.solids + s, lds, s_wave, nullptr);
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
