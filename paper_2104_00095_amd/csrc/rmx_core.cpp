// Host core of librmx: argument validation, planning of one batched call, workspace,
// the launch chain, an optional hipGraph cache, and per-solid statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "rmx.h"
#include "rmx_core.h"
#include "rmx_internal.h"

using namespace rmx;

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Sizing without a device: the largest label tile (most slot padding).
constexpr size_t kMaxLdsBytes = 160 * 1024;

// The single persistent launch took a GPU memory fault whose cause is not known; until
// it is, a library build refuses it (RMX_E_DISABLED).  Only the CPU emulation of the
// kernels, a test harness, defines RMX_ENABLE_PERSISTENT.
#ifdef RMX_ENABLE_PERSISTENT
constexpr bool kPersistentEnabled = true;
#else
constexpr bool kPersistentEnabled = false;
#endif

bool persistent_requested(const rmx_options* o) {
    return (o->flags & RMX_FLAG_PERSISTENT) && !(o->flags & RMX_FLAG_PER_SOLID);
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

bool finite_all(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

}  // namespace

// ------------------------------------------------------------------------------------
// Validation and planning (shared with the server).
// ------------------------------------------------------------------------------------
int rmx_validate(const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
                 const rmx_options* opt) {
    if (!grid || !solids || n_solids < 1 || !opt) return RMX_E_ARG;
    for (int a = 0; a < 3; ++a)
        if (grid->n[a] <= 0) return RMX_E_ARG;
    if (!(grid->h > 0.0) || !std::isfinite(grid->h) || !finite_all(grid->origin, 3))
        return RMX_E_ARG;
    if (opt->r_s < 1 || opt->r_max < opt->r_s || opt->r_max > RMX_MAX_RADIUS) return RMX_E_ARG;
    if (opt->normal_layers < 0 || opt->normal_layers > RMX_MAX_LAYERS) return RMX_E_ARG;
    if (opt->precision != RMX_FP64 && opt->precision != RMX_FP32_ACCUM) return RMX_E_ARG;
    for (int i = 0; i < n_solids; ++i) {
        const rmx_solid& s = solids[i];
        for (int a = 0; a < 3; ++a) {
            if (s.ext[a] <= 0 || s.lo[a] < 0) return RMX_E_BOX;
            if ((int64_t)s.lo[a] + s.ext[a] > grid->n[a]) return RMX_E_BOX;
        }
        const int64_t ncell = (int64_t)s.ext[0] * s.ext[1] * s.ext[2];
        if (ncell > (int64_t)0x7fffffff - 64) return RMX_E_BOX;
        if (s.n_layers < 0 || s.n_layers > RMX_MAX_LAYERS) return RMX_E_LAYERS;
        if (!s.xi || !s.labels) return RMX_E_ARG;
        const rmx_shape& sh = s.phi0;
        if (sh.kind != RMX_SPHERE && sh.kind != RMX_ELLIPSOID) return RMX_E_SHAPE;
        if (!finite_all(sh.centre, 3) || !finite_all(sh.rot, 9)) return RMX_E_SHAPE;
        const int na = sh.kind == RMX_SPHERE ? 1 : 3;
        for (int a = 0; a < na; ++a)
            if (!(sh.semi_axes[a] > 0.0) || !std::isfinite(sh.semi_axes[a])) return RMX_E_SHAPE;
        if (sh.kind == RMX_ELLIPSOID) {
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) {
                    double dot = 0.0;
                    for (int r = 0; r < 3; ++r) dot += sh.rot[r * 3 + p] * sh.rot[r * 3 + q];
                    if (std::fabs(dot - (p == q ? 1.0 : 0.0)) > 1e-9) return RMX_E_SHAPE;
                }
        }
    }
    return RMX_OK;
}

namespace {

// Dependency-respecting ticket order for the fused launch: per solid, classify the z-slabs
// middle-out; a slab is labelled once its neighbours are classified; layer l of a slab is
// fitted once its neighbours are labelled and fitted at layer l-1 (and, when the box has
// a face inside the grid, once the whole solid is classified, so that a truncated band is
// known before any write).  Solids are interleaved one classified slab at a time.
void build_items(Plan* p) {
    struct S {
        std::vector<int> order;
        size_t next = 0;
        std::vector<char> c, lb;
        std::vector<std::vector<char>> e;
        int c_left = 0;
    };
    std::vector<S> st(p->n_solids);
    for (int i = 0; i < p->n_solids; ++i) {
        const DevSolid& d = p->solids[i];
        S& x = st[i];
        const int m = d.n_slabs / 2;
        x.order.push_back(m);
        for (int k = 1; (int)x.order.size() < d.n_slabs; ++k) {
            if (m + k < d.n_slabs) x.order.push_back(m + k);
            if (m - k >= 0) x.order.push_back(m - k);
        }
        x.c.assign(d.n_slabs, 0);
        x.lb.assign(d.n_slabs, 0);
        x.e.assign(d.L + 1, std::vector<char>(d.n_slabs, 0));
        x.c_left = d.n_slabs;
    }
    auto chunks = [](const DevSolid& d, int z) {
        const int z0 = z * kTileK, z1 = std::min(z0 + kTileK, d.n2);
        const int words = (z1 - z0) * d.n1 * d.W;
        return (words + kChunkWords - 1) / kChunkWords;
    };
    p->items.clear();
    bool more = true;
    while (more) {
        more = false;
        for (int i = 0; i < p->n_solids; ++i) {
            const DevSolid& d = p->solids[i];
            S& x = st[i];
            if (x.next < x.order.size()) {
                const int z = x.order[x.next++];
                const int nch = chunks(d, z);
                for (int q = 0; q < nch; ++q)
                    p->items.push_back(FItem{FI_CLASSIFY, 0, (uint16_t)z, (uint16_t)i, (uint16_t)q});
                x.c[z] = 1;
                --x.c_left;
                more = true;
            }
            auto all3 = [&](const std::vector<char>& v, int z) {
                for (int zz = std::max(0, z - 1); zz <= std::min(d.n_slabs - 1, z + 1); ++zz)
                    if (!v[zz]) return false;
                return true;
            };
            for (int z = 0; z < d.n_slabs; ++z) {
                if (x.lb[z] || !all3(x.c, z)) continue;
                for (int q = 0; q < d.ty * d.ntx; ++q)
                    p->items.push_back(FItem{FI_LABEL, 0, (uint16_t)z, (uint16_t)i, (uint16_t)q});
                x.lb[z] = 1;
                more = true;
            }
            if (d.has_nonwall && x.c_left > 0) continue;
            for (int l = 1; l <= d.L; ++l) {
                for (int z = 0; z < d.n_slabs; ++z) {
                    if (x.e[l][z] || !all3(x.lb, z) || (l > 1 && !all3(x.e[l - 1], z))) continue;
                    for (int q = 0; q < d.parts; ++q)
                        p->items.push_back(
                            FItem{FI_EXTRAP, (uint8_t)l, (uint16_t)z, (uint16_t)i, (uint16_t)q});
                    x.e[l][z] = 1;
                    more = true;
                }
            }
        }
    }
}

}  // namespace

int rmx_plan(const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
             const rmx_options* opt, size_t lds_limit, bool fused, Plan* p) {
    // Item fields are 16-bit: very large batches or boxes take the chain.
    if (n_solids > 65535) fused = false;
    for (int i = 0; i < n_solids && fused; ++i) {
        const int slabs = (solids[i].ext[2] + kTileK - 1) / kTileK;
        const int64_t per_slab_words = (int64_t)kTileK * solids[i].ext[1] * ((solids[i].ext[0] + 63) / 64);
        if (slabs > 65535 || (per_slab_words + kChunkWords - 1) / kChunkWords > 65535 ||
            (int64_t)((solids[i].ext[1] + kTileJ - 1) / kTileJ) * ((solids[i].ext[0] + 63) / 64) > 65535)
            fused = false;
    }
    p->fused = fused;
    p->n_solids = n_solids;
    p->solids.assign(n_solids, DevSolid{});
    p->tile_solid.clear();
    p->Lmax = 0;
    int Wmax = 1;
    for (int i = 0; i < n_solids; ++i) {
        p->Lmax = std::max(p->Lmax, solids[i].n_layers);
        Wmax = std::max(Wmax, (solids[i].ext[0] + 63) / 64);
    }
    // Label tile width: as many 64-cell words as fit the LDS limit (at most 4); the fused
    // kernel uses one-word tiles (fewer registers, more and smaller items).
    int tw = fused ? 1 : std::min(4, Wmax);
    while (tw > 1 && label_lds_bytes(p->Lmax, tw, Wmax) > lds_limit) tw = tw > 2 ? 2 : 1;
    p->lds_bytes = label_lds_bytes(p->Lmax, tw, Wmax);
    if (fused) p->lds_bytes = fused_lds_bytes(p->lds_bytes);
    if (p->lds_bytes > lds_limit) return RMX_E_LAYERS;
    p->tile_w = tw;
    p->tile_cells = 64 * tw * kTileJ * kTileK;
    int64_t words = 0, slots = 0, cells = 0;
    int tiles = 0, chunks = 0;
    for (int i = 0; i < n_solids; ++i) {
        const rmx_solid& s = solids[i];
        DevSolid& d = p->solids[i];
        d.n0 = s.ext[0];
        d.n1 = s.ext[1];
        d.n2 = s.ext[2];
        d.W = (d.n0 + 63) / 64;
        d.ty = (d.n1 + kTileJ - 1) / kTileJ;
        d.tz = (d.n2 + kTileK - 1) / kTileK;
        d.L = s.n_layers;
        d.kind = s.phi0.kind;
        for (int a = 0; a < 3; ++a) {
            d.wall_lo[a] = s.lo[a] == 0;
            d.wall_hi[a] = s.lo[a] + s.ext[a] == grid->n[a];
        }
        d.ncell = (int64_t)d.n0 * d.n1 * d.n2;
        d.word_base = words;
        d.tile_base = tiles;
        d.slot_base = slots;
        d.chunk_base = chunks;
        for (int a = 0; a < 3; ++a) d.centre[a] = s.phi0.centre[a];
        if (s.phi0.kind == RMX_SPHERE) {
            d.semi[0] = d.semi[1] = d.semi[2] = s.phi0.semi_axes[0];
            for (int q = 0; q < 9; ++q) d.rot[q] = (q % 4 == 0) ? 1.0 : 0.0;
        } else {
            for (int a = 0; a < 3; ++a) d.semi[a] = s.phi0.semi_axes[a];
            for (int q = 0; q < 9; ++q) d.rot[q] = s.phi0.rot[q];
        }
        d.n_slabs = (d.n2 + kTileK - 1) / kTileK;
        d.nbx = (d.n0 + kBrick - 1) / kBrick;
        d.nby = (d.n1 + kBrick - 1) / kBrick;
        d.bcap = d.nbx * d.nby * 2;
        d.parts = std::max(4, std::min(64, d.bcap / 4));
        d.has_nonwall = 0;
        for (int a = 0; a < 3; ++a) d.has_nonwall |= !d.wall_lo[a] || !d.wall_hi[a];
        d.xi = s.xi;
        d.xi_normal = s.xi_normal ? s.xi_normal : s.xi;
        d.labels = s.labels;
        d.decisions = s.decisions;
        d.ntx = (d.W + tw - 1) / tw;
        const int nt = d.ntx * d.ty * d.tz;
        d.n_tiles = nt;
        for (int t = 0; t < nt; ++t) p->tile_solid.push_back(i);
        const int64_t nw = (int64_t)d.n1 * d.n2 * d.W;
        chunks += (int)((nw + kChunkWords - 1) / kChunkWords);
        words += nw;
        d.total_chunks = 0;
        for (int z = 0; z < d.n_slabs; ++z) {
            const int z0 = z * kTileK, z1 = std::min(z0 + kTileK, d.n2);
            d.total_chunks += ((z1 - z0) * d.n1 * d.W + kChunkWords - 1) / kChunkWords;
        }
        tiles += nt;
        slots += (int64_t)nt * p->tile_cells;
        cells += d.ncell;
    }
    p->n_tiles = tiles;
    p->n_chunks = chunks;
    p->chunk_cap = (int)(slots / kLocateChunk) + 1;
    p->total_words = words;
    p->slot_cap = slots;
    p->total_cells = cells;
    p->normal_layers = std::min(opt->normal_layers, p->Lmax);
    // Workspace layout.
    size_t off = 0;
    p->off_desc = off;
    off = align256(off + sizeof(DevSolid) * n_solids);
    p->off_tile_solid = off;
    off = align256(off + sizeof(int32_t) * tiles);
    p->desc_bytes = off;  // descriptors + tile table: one upload
    p->off_stats = off;
    off = align256(off + sizeof(unsigned long long) * kStatWords * n_solids);
    p->off_tile_cnt = off;
    off = align256(off + sizeof(int32_t) * kLT * (size_t)tiles);
    p->off_tile_lstart = off;
    off = align256(off + sizeof(int32_t) * kLT * (size_t)tiles);
    p->off_tile_off = off;
    off = align256(off + sizeof(int32_t) * kLT * (size_t)(tiles + 1));
    p->off_chunk_tile = off;
    off = align256(off + sizeof(int32_t) * kLT * (size_t)p->chunk_cap);
    p->off_chunk_flag = off;
    off = align256(off + sizeof(int32_t) * (size_t)chunks);
    p->off_mask = off;
    off = align256(off + sizeof(unsigned long long) * (size_t)words);
    if (!fused) {
        p->off_slots = off;
        off = align256(off + sizeof(int32_t) * (size_t)slots);
        p->off_normals = off;
        if (p->normal_layers > 0) off = align256(off + 3 * sizeof(double) * (size_t)slots);
    } else {
        // per-cell normals of each solid, brick lists, counters
        p->off_normals = off;
        if (p->normal_layers > 0) off = align256(off + 3 * sizeof(double) * (size_t)cells);
        int ctr = kCtrGlobal;
        int64_t list = 0;
        for (auto& d : p->solids) {
            d.ctr = ctr;
            ctr += kCtrSolid + d.n_slabs * (2 + 2 * d.L);
            d.list = list;
            list += (int64_t)d.L * d.n_slabs * d.bcap;
        }
        p->ctr_words = ctr;
        p->off_lists = off;
        off = align256(off + sizeof(int32_t) * (size_t)std::max<int64_t>(list, 1));
        build_items(p);
    }
    p->ws_bytes = off;
    return RMX_OK;
}

void rmx_bind(Plan* p, void* ws, const rmx_options* opt, Batch* b) {
    char* base = static_cast<char*>(ws);
    int64_t word = 0, cell = 0;
    for (auto& d : p->solids) {
        d.mask = reinterpret_cast<unsigned long long*>(base + p->off_mask) + word;
        word += (int64_t)d.n1 * d.n2 * d.W;
        d.normals = (p->fused && p->normal_layers > 0)
                        ? reinterpret_cast<double*>(base + p->off_normals) + 3 * cell
                        : nullptr;
        cell += d.ncell;
    }
    b->solids = reinterpret_cast<const DevSolid*>(base + p->off_desc);
    b->n_solids = p->n_solids;
    b->n_tiles = p->n_tiles;
    b->Lmax = p->Lmax;
    b->normal_layers = p->normal_layers;
    b->r_s = opt->r_s;
    b->r_max = opt->r_max;
    b->total_words = p->total_words;
    b->n_chunks = p->n_chunks;
    b->chunk_cap = p->chunk_cap;
    b->slot_cap = p->slot_cap;
    b->chunk_tile = reinterpret_cast<int32_t*>(base + p->off_chunk_tile);
    b->chunk_flag = reinterpret_cast<int32_t*>(base + p->off_chunk_flag);
    b->tile_w = p->tile_w;
    b->tile_cells = p->tile_cells;
    b->tile_solid = reinterpret_cast<const int32_t*>(base + p->off_tile_solid);
    b->tile_cnt = reinterpret_cast<int32_t*>(base + p->off_tile_cnt);
    b->tile_lstart = reinterpret_cast<int32_t*>(base + p->off_tile_lstart);
    b->tile_off = reinterpret_cast<int32_t*>(base + p->off_tile_off);
    b->slots = reinterpret_cast<int32_t*>(base + p->off_slots);
    b->normals = reinterpret_cast<double*>(base + p->off_normals);
    b->stats = reinterpret_cast<unsigned long long*>(base + p->off_stats);
}

void rmx_pack_desc(const Plan& p, void* host) {
    char* h = static_cast<char*>(host);
    std::memcpy(h + p.off_desc, p.solids.data(), sizeof(DevSolid) * p.n_solids);
    std::memcpy(h + p.off_tile_solid, p.tile_solid.data(), sizeof(int32_t) * p.n_tiles);
}

hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipError_t Profiler::begin(int phase, hipStream_t st, Rec* r) {
    r->phase = phase;
    r->a = get();
    r->b = get();
    if (!r->a || !r->b) return hipErrorOutOfMemory;
    return hipEventRecord(r->a, st);
}

hipError_t Profiler::end(Rec& r, hipStream_t st) {
    hipError_t e = hipEventRecord(r.b, st);
    pending.push_back(r);
    return e;
}

hipError_t Profiler::drain() {
    hipError_t err = hipSuccess;
    for (auto& r : pending) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) err = e;
        ms[r.phase] += t;
        launches[r.phase] += 1;
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    pending.clear();
    return err;
}

Profiler::~Profiler() {
    (void)drain();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

// The kernels of one batched call, in stream order.  Nothing here allocates or
// synchronises, so the sequence can be captured into a graph.  With a profiler, each
// launch is bracketed by HIP events on the same stream.
hipError_t rmx_enqueue(const Plan& p, const Batch& b, int precision, hipStream_t st,
                       Profiler* prof) {
    hipError_t e;
    Profiler::Rec rec{};
#define RMX_TIMED(phase, call)                                              \
    do {                                                                    \
        if (prof && (e = prof->begin((phase), st, &rec)) != hipSuccess) return e; \
        if ((e = (call)) != hipSuccess) return e;                            \
        if (prof && (e = prof->end(rec, st)) != hipSuccess) return e;        \
    } while (0)
    RMX_TIMED(RMX_PHASE_CLASSIFY, launch_classify(b, st));
    RMX_TIMED(RMX_PHASE_LABEL, launch_label(b, p.lds_bytes, st));
    RMX_TIMED(RMX_PHASE_SCAN, launch_scan(b, st));
    if (p.Lmax == 0) return hipSuccess;
    // Band cells of one layer: a thin shell; the kernels stride over the true count.
    const int64_t est = std::max<int64_t>(4096, p.total_cells / 8);
    if (p.normal_layers > 0)
        RMX_TIMED(RMX_PHASE_NORMAL, launch_normal(b, est * p.normal_layers, st));
    for (int l = 1; l <= p.Lmax; ++l)
        RMX_TIMED(RMX_PHASE_EXTRAP + l - 1, launch_extrap(b, l, precision, est, st));
#undef RMX_TIMED
    return hipSuccess;
}

void rmx_convert_stats(const unsigned long long* dev, int n, rmx_solid_stats* out) {
    for (int i = 0; i < n; ++i) {
        const unsigned long long* s = dev + (size_t)i * kStatWords;
        rmx_solid_stats& o = out[i];
        std::memset(&o, 0, sizeof(o));
        o.n_interior = (int64_t)s[ST_INTERIOR];
        for (int l = 1; l <= RMX_MAX_LAYERS; ++l) o.n_band[l] = (int64_t)s[l];
        o.n_r_grown = (int64_t)s[ST_GROWN];
        o.n_no_normal = (int64_t)s[ST_NONORMAL];
        o.n_f1 = (int64_t)s[ST_F1];
        o.n_f2 = (int64_t)s[ST_F2];
        if (s[ST_FLAGS] & FLAG_TIMEOUT)
            o.status = RMX_E_HIP;
        else if (s[ST_FLAGS] & FLAG_TRUNCATED)
            o.status = RMX_E_TRUNCATED;
        else if (o.n_interior == 0)
            o.status = RMX_W_EMPTY;
        else
            o.status = RMX_OK;
    }
}

// ------------------------------------------------------------------------------------
// Context.
// ------------------------------------------------------------------------------------
namespace {

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* ws_base = nullptr;
};

struct Staging {
    void* host = nullptr;
    size_t size = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

}  // namespace

struct rmx_ctx {
    int device = 0;
    size_t lds_limit = 65536;
    bool fixed = false;
    void* ws = nullptr;
    size_t ws_size = 0;
    static constexpr int kRing = 4;
    Staging stage[kRing];
    int stage_next = 0;
    unsigned long long* stats_host = nullptr;
    size_t stats_host_n = 0;
    hipStream_t capture_stream = nullptr;
    std::unordered_map<uint64_t, GraphEntry> graphs;
    std::vector<rmx_solid_stats> tmp_stats;
    Profiler prof;
    // fused launch: item list (cached by content), self-resetting counters, grid sizes
    FItem* items = nullptr;
    size_t items_cap = 0;
    size_t items_n = 0;
    uint64_t items_key = 0;
    int* ctr = nullptr;
    size_t ctr_cap = 0;
    std::unordered_map<uint64_t, int> fused_blocks;
};

namespace {

void drop_graphs(rmx_ctx* c);

// Upload the item list unless the cached one is identical.
int ensure_items(rmx_ctx* c, const Plan& p, hipStream_t st) {
    const size_t n = p.items.size();
    const uint64_t key = fnv1a(p.items.data(), n * sizeof(FItem), 1469598103934665603ull ^ n);
    if (c->items && c->items_n == n && c->items_key == key) return RMX_OK;
    if (n > c->items_cap) {
        if (c->items) {
            if (hipDeviceSynchronize() != hipSuccess) return RMX_E_HIP;
            drop_graphs(c);
            (void)hipFree(c->items);
            c->items = nullptr;
        }
        const size_t cap = n + n / 2 + 64;
        if (hipMalloc(&c->items, cap * sizeof(FItem)) != hipSuccess) {
            c->items = nullptr;
            c->items_cap = 0;
            return RMX_E_HIP;
        }
        c->items_cap = cap;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return RMX_E_HIP;
    if (hipMemcpy(c->items, p.items.data(), n * sizeof(FItem), hipMemcpyHostToDevice) !=
        hipSuccess)
        return RMX_E_HIP;
    c->items_n = n;
    c->items_key = key;
    return RMX_OK;
}

// Counters start at zero and the kernel's last block resets them, so a grown buffer is
// cleared once, here, outside any graph.
int ensure_ctr(rmx_ctx* c, size_t words) {
    if (words <= c->ctr_cap) return RMX_OK;
    if (c->ctr) {
        if (hipDeviceSynchronize() != hipSuccess) return RMX_E_HIP;
        drop_graphs(c);
        (void)hipFree(c->ctr);
        c->ctr = nullptr;
    }
    const size_t cap = words + words / 2 + 256;
    if (hipMalloc(&c->ctr, cap * sizeof(int)) != hipSuccess) {
        c->ctr = nullptr;
        c->ctr_cap = 0;
        return RMX_E_HIP;
    }
    if (hipMemset(c->ctr, 0, cap * sizeof(int)) != hipSuccess) return RMX_E_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return RMX_E_HIP;
    c->ctr_cap = cap;
    return RMX_OK;
}

void drop_graphs(rmx_ctx* c) {
    for (auto& kv : c->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    c->graphs.clear();
}

int ensure_ws(rmx_ctx* c, size_t need) {
    if (need <= c->ws_size) return RMX_OK;
    if (c->fixed) return RMX_E_WORKSPACE;
    if (c->ws) {
        if (hipDeviceSynchronize() != hipSuccess) return RMX_E_HIP;
        drop_graphs(c);
        (void)hipFree(c->ws);
        c->ws = nullptr;
        c->ws_size = 0;
    }
    const size_t sz = need + need / 4;
    if (hipMalloc(&c->ws, sz) != hipSuccess) {
        c->ws = nullptr;
        return RMX_E_HIP;
    }
    c->ws_size = sz;
    return RMX_OK;
}

// Pinned staging buffer for the descriptor upload; waits if the slot's previous copy is
// still in flight.
int get_stage(rmx_ctx* c, size_t bytes, Staging** out) {
    Staging& s = c->stage[c->stage_next];
    c->stage_next = (c->stage_next + 1) % rmx_ctx::kRing;
    if (s.pending) {
        if (hipEventSynchronize(s.ev) != hipSuccess) return RMX_E_HIP;
        s.pending = false;
    }
    if (s.size < bytes) {
        if (s.host) (void)hipHostFree(s.host);
        s.host = nullptr;
        const size_t sz = std::max<size_t>(bytes, 1 << 16);
        if (hipHostMalloc(&s.host, sz, hipHostMallocDefault) != hipSuccess) {
            s.host = nullptr;
            s.size = 0;
            return RMX_E_HIP;
        }
        s.size = sz;
    }
    *out = &s;
    return RMX_OK;
}

int ensure_stats_host(rmx_ctx* c, size_t n) {
    if (c->stats_host_n >= n) return RMX_OK;
    if (c->stats_host) (void)hipHostFree(c->stats_host);
    c->stats_host = nullptr;
    if (hipHostMalloc((void**)&c->stats_host, n * sizeof(unsigned long long),
                      hipHostMallocDefault) != hipSuccess) {
        c->stats_host_n = 0;
        return RMX_E_HIP;
    }
    c->stats_host_n = n;
    return RMX_OK;
}

uint64_t call_key(const rmx_grid* g, const rmx_solid* s, int n, const rmx_options* o) {
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(g, sizeof(*g), h);
    h = fnv1a(s, sizeof(*s) * (size_t)n, h);
    rmx_options oo = *o;
    oo.flags &= RMX_FLAG_PER_SOLID;
    h = fnv1a(&oo, sizeof(oo), h);
    return h;
}

// One batched call (all of `solids`) enqueued on `st`.
int run_batch(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids, int n,
              const rmx_options* opt, hipStream_t st, bool use_graph, size_t stats_off,
              bool want_stats) {
    const bool fused = persistent_requested(opt);
    Plan p;
    int rc = rmx_plan(grid, solids, n, opt, c->lds_limit, fused, &p);
    if (rc != RMX_OK) return rc;
    rc = ensure_ws(c, p.ws_bytes);
    if (rc != RMX_OK) return rc;
    Batch b{};
    rmx_bind(&p, c->ws, opt, &b);
    Fused f{};
    int blocks = 0;
    if (fused) {
        if ((rc = ensure_ctr(c, (size_t)p.ctr_words)) != RMX_OK) return rc;
        if ((rc = ensure_items(c, p, st)) != RMX_OK) return rc;
        f.items = c->items;
        f.n_items = (int32_t)p.items.size();
        f.ctr_words = p.ctr_words;
        f.ctr = c->ctr;
        f.lists = reinterpret_cast<int32_t*>(static_cast<char*>(c->ws) + p.off_lists);
        f.lds_work = (int32_t)(p.lds_bytes - kFusedSmallBytes);
        const uint64_t gkey = ((uint64_t)opt->precision << 40) ^ (uint64_t)p.lds_bytes;
        auto it = c->fused_blocks.find(gkey);
        if (it == c->fused_blocks.end()) {
            int nb = 0;
            if (fused_grid(opt->precision, p.lds_bytes, c->device, &nb) != hipSuccess)
                return RMX_E_HIP;
            it = c->fused_blocks.emplace(gkey, nb).first;
        }
        blocks = std::max(1, std::min(it->second, f.n_items));
    }
    auto enqueue = [&](hipStream_t s, Profiler* prof) -> hipError_t {
        if (!fused) return rmx_enqueue(p, b, opt->precision, s, prof);
        Profiler::Rec rec{};
        hipError_t e;
        if (prof && (e = prof->begin(RMX_PHASE_FUSED, s, &rec)) != hipSuccess) return e;
        if ((e = launch_fused(b, f, opt->precision, p.lds_bytes, blocks, s)) != hipSuccess)
            return e;
        if (prof && (e = prof->end(rec, s)) != hipSuccess) return e;
        return hipSuccess;
    };

    if (use_graph) {
        const uint64_t key = call_key(grid, solids, n, opt);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end() || it->second.ws_base != c->ws) {
            if (it != c->graphs.end()) {
                (void)hipGraphExecDestroy(it->second.exec);
                (void)hipGraphDestroy(it->second.graph);
                c->graphs.erase(it);
            }
            // Descriptors live in the workspace; a graph replays with the same workspace,
            // so they are written once, synchronously, before capture.
            std::vector<char> host(p.desc_bytes);
            rmx_pack_desc(p, host.data());
            if (hipStreamSynchronize(st) != hipSuccess) return RMX_E_HIP;
            if (hipMemcpy(c->ws, host.data(), p.desc_bytes, hipMemcpyHostToDevice) != hipSuccess)
                return RMX_E_HIP;
            GraphEntry ge;
            ge.ws_base = c->ws;
            if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) !=
                hipSuccess)
                return RMX_E_HIP;
            hipError_t e = enqueue(c->capture_stream, nullptr);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->capture_stream, &graph);
            if (e != hipSuccess || e2 != hipSuccess || !graph) return RMX_E_HIP;
            ge.graph = graph;
            if (hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return RMX_E_HIP;
            }
            it = c->graphs.emplace(key, ge).first;
        }
        if (hipGraphLaunch(it->second.exec, st) != hipSuccess) return RMX_E_HIP;
    } else {
        Staging* sg = nullptr;
        rc = get_stage(c, p.desc_bytes, &sg);
        if (rc != RMX_OK) return rc;
        rmx_pack_desc(p, sg->host);
        if (hipMemcpyAsync(c->ws, sg->host, p.desc_bytes, hipMemcpyHostToDevice, st) !=
            hipSuccess)
            return RMX_E_HIP;
        if (hipEventRecord(sg->ev, st) != hipSuccess) return RMX_E_HIP;
        sg->pending = true;
        Profiler* prof = (opt->flags & RMX_FLAG_PROFILE) ? &c->prof : nullptr;
        if (enqueue(st, prof) != hipSuccess) return RMX_E_HIP;
    }
    if (want_stats) {
        if (hipMemcpyAsync(c->stats_host + stats_off, b.stats,
                           sizeof(unsigned long long) * kStatWords * n, hipMemcpyDeviceToHost,
                           st) != hipSuccess)
            return RMX_E_HIP;
    }
    return RMX_OK;
}

}  // namespace

extern "C" {

int rmx_default_options(rmx_options* opt) {
    if (!opt) return RMX_E_ARG;
    opt->r_s = 2;
    opt->r_max = 4;
    opt->normal_layers = 2;
    opt->precision = RMX_FP64;
    opt->flags = 0;
    return RMX_OK;
}

int rmx_create(int device, size_t workspace_bytes, rmx_ctx** out) {
    if (!out) return RMX_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RMX_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return RMX_E_HIP;
    rmx_ctx* c = new rmx_ctx();
    c->device = device;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess &&
        lds > 0)
        c->lds_limit = (size_t)lds;
    for (auto& s : c->stage)
        if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
            rmx_destroy(c);
            return RMX_E_HIP;
        }
    if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        rmx_destroy(c);
        return RMX_E_HIP;
    }
    if (workspace_bytes > 0) {
        if (hipMalloc(&c->ws, workspace_bytes) != hipSuccess) {
            c->ws = nullptr;
            rmx_destroy(c);
            return RMX_E_HIP;
        }
        c->ws_size = workspace_bytes;
        c->fixed = true;
    }
    *out = c;
    return RMX_OK;
}

int rmx_destroy(rmx_ctx* c) {
    if (!c) return RMX_E_ARG;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    drop_graphs(c);
    for (auto& s : c->stage) {
        if (s.host) (void)hipHostFree(s.host);
        if (s.ev) (void)hipEventDestroy(s.ev);
    }
    if (c->stats_host) (void)hipHostFree(c->stats_host);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->items) (void)hipFree(c->items);
    if (c->ctr) (void)hipFree(c->ctr);
    if (c->ws) (void)hipFree(c->ws);
    delete c;
    return RMX_OK;
}

int rmx_workspace_size(const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
                       const rmx_options* opt, size_t* bytes) {
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    if (!bytes) return RMX_E_ARG;
    const int v = rmx_validate(grid, solids, n_solids, opt);
    if (v != RMX_OK) return v;
    size_t total = 0;
    if (opt->flags & RMX_FLAG_PER_SOLID) {
        for (int i = 0; i < n_solids; ++i) {
            Plan p;
            const int rc = rmx_plan(grid, solids + i, 1, opt, kMaxLdsBytes, false, &p);
            if (rc != RMX_OK) return rc;
            total = std::max(total, p.ws_bytes);
        }
    } else {
        Plan p;
        const int rc = rmx_plan(grid, solids, n_solids, opt, kMaxLdsBytes,
                                persistent_requested(opt), &p);
        if (rc != RMX_OK) return rc;
        total = p.ws_bytes;
    }
    *bytes = total;
    return RMX_OK;
}

int rmx_extrapolate(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids,
                    int32_t n_solids, const rmx_options* opt, void* hip_stream,
                    rmx_solid_stats* stats) {
    if (!c) return RMX_E_ARG;
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    int rc = rmx_validate(grid, solids, n_solids, opt);
    if (rc != RMX_OK) return rc;
    if (persistent_requested(opt) && !kPersistentEnabled) return RMX_E_DISABLED;
    if (hipSetDevice(c->device) != hipSuccess) return RMX_E_HIP;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const bool sync = stats || (opt->flags & RMX_FLAG_SYNC);
    const bool use_graph = (opt->flags & RMX_FLAG_GRAPH) != 0;
    if (sync) {
        rc = ensure_stats_host(c, (size_t)kStatWords * n_solids);
        if (rc != RMX_OK) return rc;
    }
    if (opt->flags & RMX_FLAG_PER_SOLID) {
        for (int i = 0; i < n_solids; ++i) {
            rc = run_batch(c, grid, solids + i, 1, opt, st, use_graph,
                           (size_t)kStatWords * i, sync);
            if (rc != RMX_OK) return rc;
        }
    } else {
        rc = run_batch(c, grid, solids, n_solids, opt, st, use_graph, 0, sync);
        if (rc != RMX_OK) return rc;
    }
    if (!sync) return RMX_OK;
    if (hipStreamSynchronize(st) != hipSuccess) return RMX_E_HIP;
    c->tmp_stats.resize(n_solids);
    rmx_convert_stats(c->stats_host, n_solids, c->tmp_stats.data());
    if (stats) std::memcpy(stats, c->tmp_stats.data(), sizeof(rmx_solid_stats) * n_solids);
    for (int i = 0; i < n_solids; ++i)
        if (c->tmp_stats[i].status < 0) return c->tmp_stats[i].status;
    return RMX_OK;
}

int rmx_profile_read(rmx_ctx* c, double* ms, int64_t* launches) {
    if (!c) return RMX_E_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return RMX_E_HIP;
    const hipError_t e = c->prof.drain();
    for (int i = 0; i < RMX_N_PHASES; ++i) {
        if (ms) ms[i] = c->prof.ms[i];
        if (launches) launches[i] = c->prof.launches[i];
        c->prof.ms[i] = 0.0;
        c->prof.launches[i] = 0;
    }
    return e == hipSuccess ? RMX_OK : RMX_E_HIP;
}

const char* rmx_status_string(int s) {
    switch (s) {
        case RMX_OK: return "ok";
        case RMX_W_EMPTY: return "no interior cell";
        case RMX_E_ARG: return "invalid argument";
        case RMX_E_BOX: return "box outside the grid";
        case RMX_E_LAYERS: return "layer count out of range";
        case RMX_E_SHAPE: return "invalid shape";
        case RMX_E_WORKSPACE: return "workspace too small";
        case RMX_E_HIP: return "HIP runtime error";
        case RMX_E_TRUNCATED: return "band truncated by the box";
        case RMX_E_BUDGET: return "request exceeds the HBM budget";
        case RMX_E_BUSY: return "queue full";
        case RMX_E_NOTFOUND: return "not found";
        case RMX_E_DISABLED: return "launch form switched off in this build";
        default: return "unknown status";
    }
}

}  // extern "C"
