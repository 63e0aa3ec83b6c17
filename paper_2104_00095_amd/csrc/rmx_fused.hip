// Fused persistent form (gfx950): every solid of a call, every phase and every layer in
// ONE launch.  Blocks take work items by ticket from an item list ordered so that each
// item's dependencies have smaller tickets; an item waits (bounded spin) on per-slab
// completion counters.  Because a ticket is only ever held by a running block, the item
// with the smallest unfinished ticket can always proceed: no deadlock, whatever the
// residency.  Classification of later z-slabs streams from HBM while the band of earlier
// slabs is labelled and fitted, so the latency-bound fits hide under the scan.
//
// Items per solid (z-slab = kTileK planes):
//   classify (slab, chunk)  one 64-word chunk of the 1-bit interior mask
//   label (slab, tile)      labels, normals of layers <= normal_layers, and the list of
//                           8^3 bricks holding cells of each layer
//   extrap (slab, layer, part)  fits of the layer's cells brick by brick: the brick and a
//                           halo of r_s = 2 cells are staged in LDS, so the r_s gather
//                           reads only LDS; grown radii and fallbacks read global memory
// Method: Lin, Derr & Rycroft (arXiv 2104.00095), section "Extrapolation of xi(x,t)";
// SI "Weighting scheme for weighted least squares-based extrapolation", eq. (weight).
#include "rmx_device.h"
#include "rmx_fused_common.h"

namespace rmx {
namespace {
using namespace dev;

constexpr int kSpinLimit = 1 << 24;   // ~ seconds of sleeping: only a safety net

__device__ __forceinline__ int load_acq(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *p >= target; false (and the call's error flag) on timeout.  Once
// the flag is set every later wait returns at once, so a fault cannot stall the launch.
__device__ __forceinline__ bool wait_ge(const int* p, int target, int* err) {
    int spins = 0;
    while (load_acq(p) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kSpinLimit || load_acq(err)) {
            atomicOr(err, 1);
            return false;
        }
    }
    return true;
}

struct SolidCtr {
    int* base;
    int n_slabs, L;
    __device__ int* call() const { return base; }
    __device__ int* trunc() const { return base + 1; }
    __device__ int* grown() const { return base + 2; }
    __device__ int* nonormal() const { return base + 3; }
    __device__ int* f1() const { return base + 4; }
    __device__ int* f2() const { return base + 5; }
    __device__ int* cls(int z) const { return base + kCtrSolid + z; }
    __device__ int* lab(int z) const { return base + kCtrSolid + n_slabs + z; }
    __device__ int* ext(int l, int z) const { return base + kCtrSolid + (2 + (l - 1)) * n_slabs + z; }
    __device__ int* nbr(int l, int z) const {
        return base + kCtrSolid + (2 + L + (l - 1)) * n_slabs + z;
    }
};

__device__ __forceinline__ SolidCtr solid_ctr(const Fused& f, const DevSolid* d) {
    SolidCtr c;
    c.base = f.ctr + d->ctr;
    c.n_slabs = d->n_slabs;
    c.L = d->L;
    return c;
}

__device__ __forceinline__ int slab_chunks(const DevSolid* d, int z) {
    const int z0 = z * kTileK, z1 = min(z0 + kTileK, d->n2);
    const int words = (z1 - z0) * d->n1 * d->W;
    return (words + kChunkWords - 1) / kChunkWords;
}

// ------------------------------------------------------------------------------------
// Extrapolation of the layer-l cells of one brick, staged in LDS.
// ------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void gather_lds(const double* __restrict__ sx,
                                           const int8_t* __restrict__ sl, int idx, int le,
                                           bool use_normal, double g0, double g1, double g2,
                                           double rgn, double a0, double a1, double a2,
                                           int lq, Moments<T>& acc) {
    constexpr int S = kBrickSpan, S2 = kBrickSpan * kBrickSpan;
#pragma unroll 1
    for (int row = lq; row < 25; row += kLanes) {
        const int dy = row % 5 - 2, dz = row / 5 - 2;
        const int rb = idx + dz * S2 + dy * S;
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const int q = rb + dx;
            const int lab = sl[q];
            double w = 0.0;
            bool e = lab >= 0 && lab < le;
            if (e) e = weight_of(dx, dy, dz, use_normal, g0, g1, g2, rgn, w);
            if (!e) continue;
            add_datum<T>(acc, (T)w, dx, dy, dz, (T)(sx[q] - a0), (T)(sx[kBrickCells + q] - a1),
                         (T)(sx[2 * kBrickCells + q] - a2), true);
        }
    }
}

template <typename T>
__device__ void extrap_brick(const Batch& b, const Fused& f, const DevSolid* d,
                             const SolidCtr& sc, int l, int bx, int by, int bz,
                             unsigned char* lds, int* s_wave) {
    double* sx = reinterpret_cast<double*>(lds);
    int8_t* sl = reinterpret_cast<int8_t*>(lds + kBrickCells * 24);
    uint16_t* cells = reinterpret_cast<uint16_t*>(lds + kBrickCells * 25);
    const int tid = threadIdx.x;
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
    const int64_t nc = d->ncell;
    const double* __restrict__ xi = d->xi;
    const int8_t* __restrict__ labels = d->labels;
    const int ox = kBrick * bx - kBrickHalo, oy = kBrick * by - kBrickHalo,
              oz = kBrick * bz - kBrickHalo;
    for (int q = tid; q < kBrickCells; q += 256) {
        const int x = q % kBrickSpan, y = (q / kBrickSpan) % kBrickSpan,
                  z = q / (kBrickSpan * kBrickSpan);
        const int gx = ox + x, gy = oy + y, gz = oz + z;
        const bool in = (unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1 &&
                        (unsigned)gz < (unsigned)n2;
        const int32_t c = in ? (gz * n1 + gy) * n0 + gx : 0;
        const int lab = labels[c];
        const double v0 = xi[c], v1 = xi[nc + c], v2 = xi[2 * nc + c];
        sl[q] = in ? (int8_t)lab : (int8_t)-1;
        sx[q] = in ? v0 : 0.0;
        sx[kBrickCells + q] = in ? v1 : 0.0;
        sx[2 * kBrickCells + q] = in ? v2 : 0.0;
    }
    __syncthreads();
    // the layer-l cells of the brick interior, compacted
    int mine[2], cnt = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = tid + 256 * h;
        const int x = kBrickHalo + q % kBrick, y = kBrickHalo + (q / kBrick) % kBrick,
                  z = kBrickHalo + q / (kBrick * kBrick);
        const int idx = (z * kBrickSpan + y) * kBrickSpan + x;
        mine[h] = sl[idx] == l ? idx : -1;
        cnt += mine[h] >= 0;
    }
    int excl, total;
    block_scan<4>(cnt, excl, total, s_wave);
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (mine[h] >= 0) cells[excl++] = (uint16_t)mine[h];
    __syncthreads();

    const int grp = tid / kLanes, lq = tid % kLanes;
    for (int ci = grp; ci < total; ci += 256 / kLanes) {
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
        // anchor: first face neighbour in a lower layer (-x, +x, -y, +y, -z, +z)
        const int nb[6] = {idx - 1, idx + 1, idx - kBrickSpan, idx + kBrickSpan,
                           idx - kBrickSpan * kBrickSpan, idx + kBrickSpan * kBrickSpan};
        const int32_t nbg[6] = {cell - 1, cell + 1, cell - n0, cell + n0, cell - n0 * n1,
                                cell + n0 * n1};
        int aidx = idx;
        cx.anchor = cell;
#pragma unroll
        for (int q = 5; q >= 0; --q) {
            const int lb = sl[nb[q]];
            if (lb >= 0 && lb < l) {
                aidx = nb[q];
                cx.anchor = nbg[q];
            }
        }
        cx.a0 = sx[aidx];
        cx.a1 = sx[kBrickCells + aidx];
        cx.a2 = sx[2 * kBrickCells + aidx];
        bool has_normal = false;
        cx.g0 = cx.g1 = cx.g2 = cx.rgn = 0.0;
        if (l <= b.normal_layers) {
            cx.g0 = d->normals[cell];
            cx.g1 = d->normals[nc + cell];
            cx.g2 = d->normals[2 * nc + cell];
            has_normal = cx.g0 != 0.0 || cx.g1 != 0.0 || cx.g2 != 0.0;
            if (has_normal) cx.rgn = 1.0 / norm3(cx.g0, cx.g1, cx.g2);
        }
        const bool no_normal = (l <= b.normal_layers) && !has_normal;

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
            if (r == kBrickHalo)
                gather_lds<T>(sx, sl, idx, l, un, cx.g0, cx.g1, cx.g2, cx.rgn, cx.a0, cx.a1,
                              cx.a2, lq, acc);
            else
                gather_any<T>(cx, r, un, lq, acc);
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
            d->xi[cell] = cx.a0 + res[0];
            d->xi[nc + cell] = cx.a1 + res[1];
            d->xi[2 * nc + cell] = cx.a2 + res[2];
            if (d->decisions) d->decisions[cell] = (int8_t)(code + (no_normal ? kDecNoNormal : 0));
            if (code == kDecF1) atomicAdd(sc.f1(), 1);
            if (code == kDecF2) atomicAdd(sc.f2(), 1);
            if (code == kDecF1 || code == kDecF2 || code > b.r_s) atomicAdd(sc.grown(), 1);
        }
    }
    __syncthreads();   // the LDS is reused by the next brick
}

// ------------------------------------------------------------------------------------
// The persistent kernel.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256, 3) void k_fused(Batch b, Fused f) {
    // One dynamic LDS allocation: the item's work area, then the block's small shared
    // state (so that nothing of the block lives in static LDS).
    HIP_DYNAMIC_SHARED(double, lds_d)
    unsigned char* lds = reinterpret_cast<unsigned char*>(lds_d);
    int* s_wave = reinterpret_cast<int*>(lds + f.lds_work);
    int& s_ticket = s_wave[4];
    int& s_last = s_wave[5];
    unsigned char* s_bflag = lds + f.lds_work + kFusedSmallInts * sizeof(int);
    const int tid = threadIdx.x;
    int* err = f.ctr + 2;
    for (;;) {
        if (tid == 0) s_ticket = atomicAdd(f.ctr, 1);
        __syncthreads();
        const int t = s_ticket;
        __syncthreads();
        if (t >= f.n_items) break;
        const FItem it = f.items[t];
        const int s = it.solid, z = it.slab, l = it.layer;
        const DevSolid* d = b.solids + s;
        const SolidCtr sc = solid_ctr(f, d);
        if (it.type == FI_CLASSIFY) {
            const int z0 = z * kTileK;
            const int wb = z0 * d->n1 * d->W + it.idx * kChunkWords;
            const int we = min(wb + kChunkWords, min(z0 + kTileK, d->n2) * d->n1 * d->W);
            const bool tr = classify_words(d, wb, we);
            const int any = __syncthreads_or(tr);
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                if (any) atomicOr(sc.trunc(), 1);
                atomicAdd(sc.cls(z), 1);
                atomicAdd(sc.call(), 1);
            }
        } else if (it.type == FI_LABEL) {
            if (tid == 0) {
                for (int zz = max(0, z - 1); zz <= min(d->n_slabs - 1, z + 1); ++zz)
                    wait_ge(sc.cls(zz), slab_chunks(d, zz), err);
            }
            __syncthreads();
            __threadfence();
            const int tile = d->tile_base + z * d->ty * d->ntx + it.idx;
            label_tile<true, 1>(b, &f, tile, s, d, lds, s_wave, s_bflag);
            __threadfence();
            __syncthreads();
            if (tid == 0) atomicAdd(sc.lab(z), 1);
        } else {
            if (tid == 0) {
                const int per_slab = d->ty * d->ntx;
                for (int zz = max(0, z - 1); zz <= min(d->n_slabs - 1, z + 1); ++zz) {
                    wait_ge(sc.lab(zz), per_slab, err);
                    if (l > 1) wait_ge(sc.ext(l - 1, zz), d->parts, err);
                }
                if (d->has_nonwall) wait_ge(sc.call(), d->total_chunks, err);
                const int tr = __hip_atomic_load(sc.trunc(), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                s_ticket = tr ? 0 : __hip_atomic_load(sc.nbr(l, z), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            __threadfence();
            const int nbk = s_ticket;   // bricks of (slab, layer); 0 if the band is truncated
            {
                const int32_t* lst = f.lists + d->list + ((int64_t)(l - 1) * d->n_slabs + z) * d->bcap;
                for (int bi = it.idx; bi < nbk; bi += d->parts) {
                    const int pk = lst[bi];
                    extrap_brick<T>(b, f, d, sc, l, pk & 1023, (pk >> 10) & 1023, pk >> 20, lds,
                                    s_wave);
                }
            }
            __threadfence();
            __syncthreads();
            if (tid == 0) atomicAdd(sc.ext(l, z), 1);
        }
    }
    // The last block to finish writes the per-solid statistics and resets the counters.
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(f.ctr + 1, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int e = load_acq(err);
    for (int s = tid; s < b.n_solids; s += 256) {
        const DevSolid* d = b.solids + s;
        const SolidCtr sc = solid_ctr(f, d);
        unsigned long long* st = b.stats + (int64_t)s * kStatWords;
        for (int l = 0; l <= kMaxLayers; ++l) {
            long long sum = 0;
            if (l <= d->L)
                for (int t = d->tile_base; t < d->tile_base + d->n_tiles; ++t)
                    sum += b.tile_cnt[t * kLT + l];
            st[l] = (unsigned long long)sum;
        }
        st[ST_GROWN] = (unsigned long long)*sc.grown();
        st[ST_NONORMAL] = (unsigned long long)*sc.nonormal();
        st[ST_F1] = (unsigned long long)*sc.f1();
        st[ST_F2] = (unsigned long long)*sc.f2();
        st[ST_FLAGS] = (*sc.trunc() ? FLAG_TRUNCATED : 0ull) | (e ? FLAG_TIMEOUT : 0ull);
        for (int q = ST_FLAGS + 1; q < kStatWords; ++q) st[q] = 0ull;
    }
    __syncthreads();
    for (int q = tid; q < f.ctr_words; q += 256) f.ctr[q] = 0;
}

}  // namespace

size_t fused_lds_bytes(size_t label_lds) {
    const size_t work = label_lds > kBrickLds ? label_lds : kBrickLds;
    return work + kFusedSmallBytes;
}

hipError_t fused_grid(int precision, size_t lds, int device, int* blocks) {
    int per_cu = 0, cus = 0;
    hipError_t e;
    if (precision == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<float>, 256, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<double>, 256, lds);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    *blocks = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    return hipSuccess;
}

hipError_t launch_fused(const Batch& b, const Fused& f, int precision, size_t lds, int blocks,
                        hipStream_t st) {
    if (precision == 1)
        hipLaunchKernelGGL(k_fused<float>, dim3(blocks), dim3(256), lds, st, b, f);
    else
        hipLaunchKernelGGL(k_fused<double>, dim3(blocks), dim3(256), lds, st, b, f);
    return hipGetLastError();
}

}  // namespace rmx
