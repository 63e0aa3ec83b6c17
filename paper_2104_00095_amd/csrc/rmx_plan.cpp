// Validation, planning (tiles, chunks, bricks, workspace layout) and the launch sequence
// of one batched call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "rmx_core.h"

namespace rmx {
namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// End of a workspace region of `bytes` starting at `off`: the next region's start.  The
// CPU emulation build leaves a red zone after every region and records it, so that an
// access running past a region is caught there; the library build packs them.
#ifdef RMX_EMU_REDZONES
constexpr size_t kRedZone = 4096;
#else
constexpr size_t kRedZone = 0;
#endif

size_t next_region(Plan* p, size_t off, size_t bytes) {
    const size_t end = off + bytes;
    if (kRedZone) p->gaps.push_back({(end + 7) & ~size_t(7), kRedZone});
    return align256(end + kRedZone);
}

bool finite_all(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// Bricks along an axis are packed in 10 bits of a brick-list entry.
constexpr int kMaxExtent = 1023 * kBrick;

}  // namespace

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

int validate_options(const rmx_options* opt) {
    if (!opt) return RMX_E_ARG;
    if (opt->r_s < 1 || opt->r_max < opt->r_s || opt->r_max > RMX_MAX_RADIUS) return RMX_E_ARG;
    if (opt->normal_layers < 0 || opt->normal_layers > RMX_MAX_LAYERS) return RMX_E_ARG;
    if (opt->precision != RMX_FP64 && opt->precision != RMX_FP32_ACCUM) return RMX_E_ARG;
    return RMX_OK;
}

int validate_solid(const rmx_grid* grid, const rmx_solid* sp, bool need_fields) {
    if (!grid || !sp) return RMX_E_ARG;
    for (int a = 0; a < 3; ++a)
        if (grid->n[a] <= 0) return RMX_E_ARG;
    if (!(grid->h > 0.0) || !std::isfinite(grid->h) || !finite_all(grid->origin, 3))
        return RMX_E_ARG;
    for (int a = 0; a < 3; ++a)
        if (!(grid->spacing[a] >= 0.0) || !std::isfinite(grid->spacing[a])) return RMX_E_ARG;
    if (grid->reserved != 0) return RMX_E_ARG;
    const rmx_solid& s = *sp;
    for (int a = 0; a < 3; ++a) {
        if (s.ext[a] <= 0 || s.lo[a] < 0 || s.ext[a] > kMaxExtent) return RMX_E_BOX;
        if (grid->periodic[a]) {
            // the box starts on the grid and may wrap, but covers no cell twice
            if (s.lo[a] >= grid->n[a] || s.ext[a] > grid->n[a]) return RMX_E_BOX;
        } else if ((int64_t)s.lo[a] + s.ext[a] > grid->n[a]) {
            return RMX_E_BOX;
        }
    }
    const int64_t ncell = (int64_t)s.ext[0] * s.ext[1] * s.ext[2];
    if (ncell > (int64_t)0x7fffffff - 64) return RMX_E_BOX;
    if (s.n_layers < 0 || s.n_layers > RMX_MAX_LAYERS) return RMX_E_LAYERS;
    if (need_fields && (!s.xi || !s.labels)) return RMX_E_ARG;
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
    return RMX_OK;
}

int plan(const rmx_grid* const* grids, const rmx_solid* solids, int32_t n_solids,
         const rmx_options* opt, size_t lds_limit, int cu, const Tuning& tune, Plan* p,
         int normal_per_cu, int band_per_cu, int normal_sphere_per_cu) {
    p->n_solids = n_solids;
    p->solids.assign(n_solids, DevSolid{});
    p->tile_solid.clear();
    p->gaps.clear();
    p->Lmax = 0;
    int Wmax = 1;
    for (int i = 0; i < n_solids; ++i) {
        p->Lmax = std::max(p->Lmax, solids[i].n_layers);
        Wmax = std::max(Wmax, (solids[i].ext[0] + 63) / 64);
    }
    // Label tile width: the tuned one, else the widest useful one; narrowed until the
    // region fits the LDS.
    int tw = tune.tile_w;
    if (tw != 1 && tw != 2 && tw != 4) tw = Wmax >= 3 ? 4 : (Wmax == 2 ? 2 : 1);
    while (tw > 1 && label_lds_bytes(p->Lmax, tw, Wmax) > lds_limit) tw /= 2;
    p->lds_bytes = label_lds_bytes(p->Lmax, tw, Wmax);
    if (p->lds_bytes > lds_limit || brick_lds_bytes(0) > lds_limit) return RMX_E_LAYERS;
    p->tile_w = tw;
    int64_t words = 0, cells = 0;
    int tiles = 0, chunks = 0;
    for (int i = 0; i < n_solids; ++i) {
        const rmx_solid& s = solids[i];
        const rmx_grid* g = grids[i];
        DevSolid& d = p->solids[i];
        d.n0 = s.ext[0];
        d.n1 = s.ext[1];
        d.n2 = s.ext[2];
        d.W = (d.n0 + 63) / 64;
        d.ty = (d.n1 + kTileJ - 1) / kTileJ;
        d.tz = (d.n2 + kTileK - 1) / kTileK;
        d.L = s.n_layers;
        d.kind = s.phi0.kind;
        for (int a = 0; a < 3; ++a) {   // a periodic axis has no walls
            d.wall_lo[a] = !g->periodic[a] && s.lo[a] == 0;
            d.wall_hi[a] = !g->periodic[a] && s.lo[a] + s.ext[a] == g->n[a];
        }
        // spacing ratios for the normal factor of eq. (weight)
        double sp[3], smin = 0.0;
        for (int a = 0; a < 3; ++a) {
            sp[a] = g->spacing[a] > 0.0 ? g->spacing[a] : g->h;
            smin = a == 0 ? sp[0] : std::min(smin, sp[a]);
        }
        d.aniso = !(sp[0] == sp[1] && sp[1] == sp[2]);
        for (int a = 0; a < 3; ++a) {
            d.rho[a] = d.aniso ? sp[a] / smin : 1.0;
            d.irho[a] = d.aniso ? 1.0 / d.rho[a] : 1.0;
        }
        d.ncell = (int64_t)d.n0 * d.n1 * d.n2;
        d.word_base = words;
        d.tile_base = tiles;
        d.chunk_base = chunks;
        d.nbx = (d.n0 + kBrick - 1) / kBrick;
        d.nby = (d.n1 + kBrick - 1) / kBrick;
        d.nbz = (d.n2 + kBrick - 1) / kBrick;
        for (int a = 0; a < 3; ++a) d.centre[a] = s.phi0.centre[a];
        if (s.phi0.kind == RMX_SPHERE) {
            d.semi[0] = d.semi[1] = d.semi[2] = s.phi0.semi_axes[0];
            for (int q = 0; q < 9; ++q) d.rot[q] = (q % 4 == 0) ? 1.0 : 0.0;
        } else {
            for (int a = 0; a < 3; ++a) d.semi[a] = s.phi0.semi_axes[a];
            for (int q = 0; q < 9; ++q) d.rot[q] = s.phi0.rot[q];
        }
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
        tiles += nt;
        cells += d.ncell;
    }
    p->n_tiles = tiles;
    p->n_chunks = chunks;
    p->total_words = words;
    p->total_cells = cells;
    // A tile lists at most 32 bricks per 64-cell word and layer (2 x 2 x 8).
    p->blist_cap = (int64_t)tiles * 32 * tw;
    p->normal_layers = std::min(opt->normal_layers, p->Lmax);
    // Blocks striding over the brick lists: no more than the bricks a list can hold (a
    // layer's list holds each brick of the boxes at most once).
    int64_t bricks = 0;
    for (const DevSolid& d : p->solids) bricks += (int64_t)d.nbx * d.nby * d.nbz;
    const int eb = tune.extrap_blocks > 0 ? tune.extrap_blocks : 3 * std::max(cu, 1);
    p->extrap_blocks = (int)std::max<int64_t>(std::min<int64_t>(eb, bricks), 1);
    p->dlist_cap = std::max<int64_t>(bricks, 1);
    // normal: as many blocks as are resident at once (each block scans the brick lists
    // once, then strides over its bricks), no more than the bricks of its layers
    p->spheres = true;
    for (const DevSolid& d : p->solids) p->spheres = p->spheres && d.kind == 1;
    const int npc = p->spheres && normal_sphere_per_cu > 0 ? normal_sphere_per_cu : normal_per_cu;
    p->normal_blocks = (int)std::max<int64_t>(
        std::min<int64_t>((int64_t)std::max(npc, 1) * std::max(cu, 1),
                          bricks * std::max(p->normal_layers, 1)),
        1);
    // persistent band launch: the resident blocks (at least one per queue)
    p->persistent = (opt->flags & RMX_FLAG_PERSISTENT) != 0;
    p->band_blocks = std::max(std::max(band_per_cu, 1) * std::max(cu, 1), kXcds);
    if (p->persistent && band_lds_bytes(opt->precision) > lds_limit) return RMX_E_LAYERS;

    // Workspace layout.
    size_t off = 0;
    p->off_desc = off;
    off = next_region(p, off, sizeof(DevSolid) * n_solids);
    p->off_tile_solid = off;
    off = next_region(p, off, sizeof(int32_t) * tiles);
    p->desc_bytes = off;  // descriptors + tile table: one upload
    p->gaps.clear();      // (the upload covers its own red zones)
    p->off_stats = off;
    off = next_region(p, off, sizeof(unsigned long long) * kStatWords * n_solids);
    p->off_tile_cnt = off;
    off = next_region(p, off, sizeof(int32_t) * kLT * (size_t)tiles);
    p->off_bcount = off;
    off = next_region(p, off, sizeof(int32_t) * kMaxLayers * kBuckets);
    p->off_mask = off;
    off = next_region(p, off, sizeof(unsigned long long) * (size_t)words);
    p->off_normals = off;
    if (p->normal_layers > 0) off = next_region(p, off, 3 * sizeof(double) * (size_t)cells);
    p->off_blist = off;
    off = next_region(p, off, sizeof(unsigned long long) * (size_t)std::max(p->Lmax, 1) *
                                  (size_t)p->blist_cap);
    p->off_dcount = off;
    off = next_region(p, off, sizeof(int32_t) * kMaxLayers);
    p->off_dlist = off;
    off = next_region(p, off, sizeof(unsigned long long) * (size_t)std::max(p->Lmax, 1) *
                                  (size_t)p->dlist_cap);
    p->off_band = off;
    off = next_region(p, off, sizeof(BandCtl));
    p->ws_bytes = off;
    return RMX_OK;
}

void bind(Plan* p, void* ws, const rmx_options* opt, Batch* b) {
    char* base = static_cast<char*>(ws);
    int64_t word = 0, cell = 0;
    for (auto& d : p->solids) {
        d.mask = reinterpret_cast<unsigned long long*>(base + p->off_mask) + word;
        word += (int64_t)d.n1 * d.n2 * d.W;
        d.normals = p->normal_layers > 0
                        ? reinterpret_cast<double*>(base + p->off_normals) + 3 * cell
                        : nullptr;
        cell += d.ncell;
    }
    *b = Batch{};
    b->solids = reinterpret_cast<const DevSolid*>(base + p->off_desc);
    b->n_solids = p->n_solids;
    b->n_tiles = p->n_tiles;
    b->Lmax = p->Lmax;
    b->normal_layers = p->normal_layers;
    b->r_s = opt->r_s;
    b->r_max = opt->r_max;
    b->tile_w = p->tile_w;
    b->adj26 = (opt->flags & RMX_FLAG_ADJ26) != 0;
    b->spheres = p->spheres ? 1 : 0;
    b->n_chunks = p->n_chunks;
    b->total_words = p->total_words;
    b->blist_cap = p->blist_cap;
    b->tile_solid = reinterpret_cast<const int32_t*>(base + p->off_tile_solid);
    b->stats = reinterpret_cast<unsigned long long*>(base + p->off_stats);
    b->tile_cnt = reinterpret_cast<int32_t*>(base + p->off_tile_cnt);
    b->bcount = reinterpret_cast<int32_t*>(base + p->off_bcount);
    b->blist = reinterpret_cast<unsigned long long*>(base + p->off_blist);
    b->dlist_cap = p->dlist_cap;
    b->dcount = reinterpret_cast<int32_t*>(base + p->off_dcount);
    b->dlist = reinterpret_cast<unsigned long long*>(base + p->off_dlist);
    b->band = reinterpret_cast<BandCtl*>(base + p->off_band);
}

void pack_desc(const Plan& p, void* host) {
    char* h = static_cast<char*>(host);
    std::memset(h, 0, p.desc_bytes);
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
hipError_t enqueue(const Plan& p, const Batch& b, int precision, hipStream_t st,
                   Profiler* prof, bool classify) {
    hipError_t e;
    Profiler::Rec rec{};
#define RMX_TIMED(phase, call)                                              \
    do {                                                                    \
        if (prof && (e = prof->begin((phase), st, &rec)) != hipSuccess) return e; \
        if ((e = (call)) != hipSuccess) return e;                            \
        if (prof && (e = prof->end(rec, st)) != hipSuccess) return e;        \
    } while (0)
    if (classify) RMX_TIMED(RMX_PHASE_CLASSIFY, launch_classify(b, st));
    RMX_TIMED(RMX_PHASE_LABEL, launch_label(b, p.lds_bytes, st));
    if (p.persistent) {
        RMX_TIMED(RMX_PHASE_BAND, launch_band(b, precision, p.band_blocks, st));
        return hipSuccess;
    }
    RMX_TIMED(RMX_PHASE_NORMAL, launch_normal(b, p.normal_blocks, st));
    for (int l = 1; l <= p.Lmax; ++l)
        RMX_TIMED(RMX_PHASE_EXTRAP + l - 1, launch_extrap(b, l, precision, p.extrap_blocks, st));
#undef RMX_TIMED
    return hipSuccess;
}

void convert_stats(const unsigned long long* dev, int n, rmx_solid_stats* out) {
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
        if (s[ST_FLAGS] & (FLAG_OVERFLOW | FLAG_TIMEOUT))
            o.status = RMX_E_HIP;
        else if (s[ST_FLAGS] & FLAG_TRUNCATED)
            o.status = RMX_E_TRUNCATED;
        else if (o.n_interior == 0)
            o.status = RMX_W_EMPTY;
        else
            o.status = RMX_OK;
    }
}

}  // namespace rmx
