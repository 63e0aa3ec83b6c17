// The context API of librmx: workspace, descriptor upload, graph cache, profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "rmx.h"
#include "rmx_core.h"
#include "rmx_ctx.h"
#include "rmx_internal.h"
#include "rmx_blur.h"

using namespace rmx;

namespace {

// Sizing without a device: the LDS of the largest gfx950 workgroup.
constexpr size_t kMaxLdsBytes = 160 * 1024;
constexpr int kDefaultCus = 256;

// Workspace of the allocation-free entry point (rmx_extrapolate_noalloc): one array per
// device the library runs on, held until the process ends, shared by every such call on
// that device (calls that overlap on one device race on it).  In host code `scratch` is
// a host-side stand-in for the symbol, not device memory: its device address is taken
// once per device, with that device current (scratch_address, from rmx_create), and
// only that address is ever passed to kernels or copies.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Pinned host buffers a context allocates at creation, so that the allocation-free entry
// point finds them in place: descriptor staging slots and per-solid statistics.
constexpr size_t kStageBytes = size_t(256) << 10;
constexpr int kPreallocStatsSolids = 4096;

int scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return RMX_E_ARG;
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return RMX_E_HIP;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
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
        c->desc_valid = false;
    }
    const size_t sz = c->exact_ws ? need : need + need / 4;
    if (hipMalloc(&c->ws, sz) != hipSuccess) {
        c->ws = nullptr;
        return RMX_E_HIP;
    }
    c->ws_size = sz;
    return RMX_OK;
}

// Pinned staging buffer for the descriptor upload; waits if the slot's previous copy is
// still in flight.  no_alloc: a slot smaller than `bytes` is an error, not a reallocation.
int get_stage(rmx_ctx* c, size_t bytes, Staging** out, bool no_alloc = false) {
    Staging& s = c->stage[c->stage_next];
    c->stage_next = (c->stage_next + 1) % rmx_ctx::kRing;
    if (s.pending) {
        if (hipEventSynchronize(s.ev) != hipSuccess) return RMX_E_HIP;
        s.pending = false;
    }
    if (s.size < bytes) {
        if (no_alloc) return RMX_E_WORKSPACE;
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

uint64_t options_key(const rmx_options* o) {
    rmx_options oo = *o;
    oo.flags &= RMX_FLAG_PER_SOLID | RMX_FLAG_ADJ26;
    return fnv1a(&oo, sizeof(oo), 1469598103934665603ull);
}

bool desc_current(const rmx_ctx* c, const void* ws, uint64_t h, size_t len) {
    return c->desc_valid && c->desc_ws == ws && c->desc_hash == h && c->desc_len == len;
}

void desc_mark(rmx_ctx* c, const void* ws, uint64_t h, size_t len) {
    c->desc_valid = true;
    c->desc_ws = ws;
    c->desc_hash = h;
    c->desc_len = len;
}

}  // namespace

namespace rmx {

int ctx_stats_host(rmx_ctx* c, size_t n) {
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

uint64_t tune_key(const Plan& p) {
    // Calls of one shape class share launch shapes: layers, row width and a size class.
    int Wmax = 1;
    for (const auto& d : p.solids) Wmax = std::max(Wmax, d.W);
    int size_class = 0;
    for (int64_t c = p.total_cells; c > 1; c >>= 2) ++size_class;
    return ((uint64_t)p.Lmax << 32) ^ ((uint64_t)Wmax << 16) ^ (uint64_t)size_class ^
           ((uint64_t)p.normal_layers << 48);
}

int plan_call(rmx_ctx* c, const rmx_grid* const* grids, const rmx_solid* solids, int n,
              const rmx_options* opt, const Tuning* force, Plan* p) {
    const int bpc = c->band_per_cu[opt->precision == RMX_FP32_ACCUM ? 1 : 0];
    int rc = plan(grids, solids, n, opt, c->lds_limit, c->cus, Tuning{}, p, c->normal_per_cu, bpc,
                  c->normal_sphere_per_cu);
    if (rc != RMX_OK) return rc;
    Tuning tn{};
    if (force) {
        tn = *force;
    } else {
        const auto it = c->tuned.find(tune_key(*p));
        if (it != c->tuned.end()) tn = it->second;
    }
    if (tn.tile_w || tn.extrap_blocks)
        rc = plan(grids, solids, n, opt, c->lds_limit, c->cus, tn, p, c->normal_per_cu, bpc,
                  c->normal_sphere_per_cu);
    return rc;
}

// A time step's launches: transverse faces, predictor (with the interior mask), the
// extrapolation chain from the labels on, corrector.
static hipError_t step_chain(const Plan& p, const Batch& b, const StepBatch& sb, int precision,
                             hipStream_t st, Profiler* prof) {
    hipError_t e;
    Profiler::Rec rec{};
    auto timed = [&](int phase, auto&& launch) -> hipError_t {
        if (prof && (e = prof->begin(phase, st, &rec)) != hipSuccess) return e;
        if ((e = launch()) != hipSuccess) return e;
        if (prof && (e = prof->end(rec, st)) != hipSuccess) return e;
        return hipSuccess;
    };
    if ((e = timed(RMX_PHASE_STEP_TRANS, [&] {
             const hipError_t r = launch_step_scan(sb, 0, st);
             return r != hipSuccess ? r : launch_step_trans(sb, st);
         })) != hipSuccess)
        return e;
    if ((e = timed(RMX_PHASE_STEP_FACES, [&] { return launch_step_faces(sb, st); })) !=
        hipSuccess)
        return e;
    if ((e = timed(RMX_PHASE_STEP_PREDICT, [&] { return launch_step_predict(sb, st); })) !=
        hipSuccess)
        return e;
    if ((e = enqueue(p, b, precision, st, prof, false)) != hipSuccess) return e;
    return timed(RMX_PHASE_STEP_CORRECT, [&] {
        const hipError_t r = launch_step_scan(sb, 1, st);
        return r != hipSuccess ? r : launch_step_correct(sb, st);
    });
}

int launch_planned(rmx_ctx* c, Plan& p, int n, const rmx_options* opt, hipStream_t st,
                   bool use_graph, size_t stats_off, bool want_stats, void* ws, size_t ws_size,
                   bool no_alloc, const StepBatch* step) {
    if (p.ws_bytes > ws_size) return RMX_E_WORKSPACE;
    if (step && use_graph) return RMX_E_ARG;
    int rc = RMX_OK;
    Batch b{};
    bind(&p, ws, opt, &b);
#ifdef RMX_EMU_REDZONES
    rmx_emu_poison_gaps(ws, ws_size, p.gaps);
#endif
    c->desc_host.resize(p.desc_bytes);
    pack_desc(p, c->desc_host.data());
    const uint64_t dh = fnv1a(c->desc_host.data(), p.desc_bytes, 1469598103934665603ull);

    if (use_graph) {
        // the descriptors (boxes, walls, shapes, field pointers) and the options fix
        // every kernel argument of the chain
        const uint64_t key = options_key(opt) ^ (dh * 31u) ^
                             ((uint64_t)p.tile_w << 56) ^ ((uint64_t)p.extrap_blocks << 40);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end() || it->second.ws_base != ws) {
            if (it != c->graphs.end()) {
                (void)hipGraphExecDestroy(it->second.exec);
                (void)hipGraphDestroy(it->second.graph);
                c->graphs.erase(it);
            }
            // Descriptors live in the workspace; a graph replays with the same workspace,
            // so they are written once, synchronously, before capture.
            if (hipStreamSynchronize(st) != hipSuccess) return RMX_E_HIP;
            if (hipMemcpy(ws, c->desc_host.data(), p.desc_bytes, hipMemcpyHostToDevice) !=
                hipSuccess)
                return RMX_E_HIP;
            desc_mark(c, ws, dh, p.desc_bytes);
            GraphEntry ge;
            ge.ws_base = ws;
            if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) !=
                hipSuccess)
                return RMX_E_HIP;
            hipError_t e = enqueue(p, b, opt->precision, c->capture_stream, nullptr);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->capture_stream, &graph);
            if (e != hipSuccess || e2 != hipSuccess || !graph) return RMX_E_HIP;
            ge.graph = graph;
            if (hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return RMX_E_HIP;
            }
            it = c->graphs.emplace(key, ge).first;
        } else if (!desc_current(c, ws, dh, p.desc_bytes)) {
            // another call rewrote the descriptors since the capture: restore them
            if (hipStreamSynchronize(st) != hipSuccess) return RMX_E_HIP;
            if (hipMemcpy(ws, c->desc_host.data(), p.desc_bytes, hipMemcpyHostToDevice) !=
                hipSuccess)
                return RMX_E_HIP;
            desc_mark(c, ws, dh, p.desc_bytes);
        }
        if (hipGraphLaunch(it->second.exec, st) != hipSuccess) return RMX_E_HIP;
    } else {
        // Upload the descriptors unless the workspace already holds these exact bytes
        // (calls on one context are ordered on one stream).
        if (!desc_current(c, ws, dh, p.desc_bytes)) {
            Staging* sg = nullptr;
            rc = get_stage(c, p.desc_bytes, &sg, no_alloc);
            if (rc != RMX_OK) return rc;
            std::memcpy(sg->host, c->desc_host.data(), p.desc_bytes);
            if (hipMemcpyAsync(ws, sg->host, p.desc_bytes, hipMemcpyHostToDevice, st) !=
                hipSuccess)
                return RMX_E_HIP;
            if (hipEventRecord(sg->ev, st) != hipSuccess) return RMX_E_HIP;
            sg->pending = true;
            desc_mark(c, ws, dh, p.desc_bytes);
        }
        Profiler* prof = (opt->flags & RMX_FLAG_PROFILE) ? &c->prof : nullptr;
        if (step) {
            StepBatch sb = *step;
            sb.solids = b.solids;
            sb.n_solids = b.n_solids;
            sb.total_words = b.total_words;
            sb.stats = b.stats;
            sb.bcount = b.bcount;
            sb.band = b.band;
            if (step_chain(p, b, sb, opt->precision, st, prof) != hipSuccess) return RMX_E_HIP;
        } else if (enqueue(p, b, opt->precision, st, prof) != hipSuccess) {
            return RMX_E_HIP;
        }
    }
    if (want_stats) {
        if (hipMemcpyAsync(c->stats_host + stats_off, b.stats,
                           sizeof(unsigned long long) * kStatWords * n, hipMemcpyDeviceToHost,
                           st) != hipSuccess)
            return RMX_E_HIP;
    }
    return RMX_OK;
}

int finish_sync(rmx_ctx* c, hipStream_t st, int n_solids, rmx_solid_stats* stats) {
    if (hipStreamSynchronize(st) != hipSuccess) return RMX_E_HIP;
    c->tmp_stats.resize(n_solids);
    convert_stats(c->stats_host, n_solids, c->tmp_stats.data());
    if (stats) std::memcpy(stats, c->tmp_stats.data(), sizeof(rmx_solid_stats) * n_solids);
    for (int i = 0; i < n_solids; ++i)
        if (c->tmp_stats[i].status < 0) return c->tmp_stats[i].status;
    return RMX_OK;
}

int run_batch(rmx_ctx* c, const rmx_grid* const* grids, const rmx_solid* solids, int n,
              const rmx_options* opt, hipStream_t st, bool use_graph, size_t stats_off,
              bool want_stats, const Tuning* force) {
    Plan p;
    int rc = plan_call(c, grids, solids, n, opt, force, &p);
    if (rc != RMX_OK) return rc;
    rc = ensure_ws(c, p.ws_bytes);
    if (rc != RMX_OK) return rc;
    return launch_planned(c, p, n, opt, st, use_graph, stats_off, want_stats, c->ws,
                          c->ws_size, false);
}

}  // namespace rmx

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
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess && v > 0)
        c->lds_limit = (size_t)v;
    v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) ==
            hipSuccess && v > 0)
        c->cus = v;
    c->normal_per_cu = normal_blocks_per_cu(false);
    c->normal_sphere_per_cu = normal_blocks_per_cu(true);
    c->band_per_cu[0] = band_blocks_per_cu(RMX_FP64);
    c->band_per_cu[1] = band_blocks_per_cu(RMX_FP32_ACCUM);
    for (auto& s : c->stage)
        if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
            rmx_destroy(c);
            return RMX_E_HIP;
        }
    if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        rmx_destroy(c);
        return RMX_E_HIP;
    }
    // Set-up of the allocation-free entry point: this device's scratch address (device
    // current), fixed-size pinned staging slots and statistics.
    if (scratch_address(device, &c->scratch) != RMX_OK ||
        ctx_stats_host(c, (size_t)kStatWords * kPreallocStatsSolids) != RMX_OK) {
        rmx_destroy(c);
        return RMX_E_HIP;
    }
    for (auto& s : c->stage) {
        if (hipHostMalloc(&s.host, kStageBytes, hipHostMallocDefault) != hipSuccess) {
            s.host = nullptr;
            rmx_destroy(c);
            return RMX_E_HIP;
        }
        s.size = kStageBytes;
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
    if (c->ws) (void)hipFree(c->ws);
    if (c->step_ws) (void)hipFree(c->step_ws);
    if (c->blur_ws) (void)hipFree(c->blur_ws);
    delete c;
    return RMX_OK;
}

int rmx_workspace_size(const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
                       const rmx_options* opt, size_t* bytes) {
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    if (!bytes || !grid || !solids || n_solids < 1) return RMX_E_ARG;
    int rc = validate_options(opt);
    if (rc != RMX_OK) return rc;
    for (int i = 0; i < n_solids; ++i)
        if ((rc = validate_solid(grid, solids + i, false)) != RMX_OK) return rc;
    size_t total = 0;
    const bool per_solid = (opt->flags & RMX_FLAG_PER_SOLID) != 0;
    const int calls = per_solid ? n_solids : 1;
    const int per_call = per_solid ? 1 : n_solids;
    std::vector<const rmx_grid*> grids(per_call, grid);
    for (int i = 0; i < calls; ++i) {
        Plan p;
        rc = plan(grids.data(), solids + i, per_call, opt, kMaxLdsBytes, kDefaultCus, Tuning{},
                  &p);
        if (rc != RMX_OK) return rc;
        total = std::max(total, p.ws_bytes);
    }
    *bytes = total;
    return RMX_OK;
}

int rmx_extrapolate(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids,
                    int32_t n_solids, const rmx_options* opt, void* hip_stream,
                    rmx_solid_stats* stats) {
    if (!c || !grid || !solids || n_solids < 1) return RMX_E_ARG;
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    int rc = validate_options(opt);
    if (rc != RMX_OK) return rc;
    for (int i = 0; i < n_solids; ++i)
        if ((rc = validate_solid(grid, solids + i)) != RMX_OK) return rc;
    if (hipSetDevice(c->device) != hipSuccess) return RMX_E_HIP;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const bool sync = stats || (opt->flags & RMX_FLAG_SYNC);
    const bool use_graph = (opt->flags & RMX_FLAG_GRAPH) != 0;
    if (sync) {
        rc = ctx_stats_host(c, (size_t)kStatWords * n_solids);
        if (rc != RMX_OK) return rc;
    }
    c->grid_ptrs.assign(n_solids, grid);
    if (opt->flags & RMX_FLAG_PER_SOLID) {
        for (int i = 0; i < n_solids; ++i) {
            rc = run_batch(c, c->grid_ptrs.data() + i, solids + i, 1, opt, st, use_graph,
                           (size_t)kStatWords * i, sync, nullptr);
            if (rc != RMX_OK) return rc;
        }
    } else {
        rc = run_batch(c, c->grid_ptrs.data(), solids, n_solids, opt, st, use_graph, 0, sync,
                       nullptr);
        if (rc != RMX_OK) return rc;
    }
    if (!sync) return RMX_OK;
    return finish_sync(c, st, n_solids, stats);
}

int rmx_step(rmx_ctx* c, const rmx_grid* grid, const rmx_step_solid* ss, int32_t n_solids,
             const rmx_options* opt, double dt, void* hip_stream, rmx_solid_stats* stats) {
    if (!c || !grid || !ss || n_solids < 1) return RMX_E_ARG;
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    int rc = validate_options(opt);
    if (rc != RMX_OK) return rc;
    if (opt->flags & (RMX_FLAG_GRAPH | RMX_FLAG_PER_SOLID | RMX_FLAG_PERSISTENT))
        return RMX_E_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt)) return RMX_E_ARG;
    // The extrapolation part works on xi^{n+1} and the labels of step n + 1.
    std::vector<rmx_solid> sol(n_solids);
    for (int i = 0; i < n_solids; ++i) {
        const rmx_step_solid& t = ss[i];
        if (!t.xi_n || !t.labels_n || !t.u || !t.uf[0] || !t.uf[1] || !t.uf[2] ||
            !t.xi_next || !t.labels_next || !t.xi_half)
            return RMX_E_ARG;
        if (t.xi_n == t.xi_next || t.xi_n == t.xi_half || t.xi_next == t.xi_half)
            return RMX_E_ARG;
        rmx_solid& s = sol[i];
        s = rmx_solid{};
        for (int a = 0; a < 3; ++a) {
            s.lo[a] = t.lo[a];
            s.ext[a] = t.ext[a];
        }
        s.phi0 = t.phi0;
        s.n_layers = t.n_layers;
        s.xi = t.xi_next;
        s.xi_normal = nullptr;
        s.labels = t.labels_next;
        s.decisions = t.decisions;
        if ((rc = validate_solid(grid, &s)) != RMX_OK) return rc;
        if (t.n_layers < 5) return RMX_E_LAYERS;
    }
    if (hipSetDevice(c->device) != hipSuccess) return RMX_E_HIP;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const bool sync = stats || (opt->flags & RMX_FLAG_SYNC);
    if (sync && (rc = ctx_stats_host(c, (size_t)kStatWords * n_solids)) != RMX_OK) return rc;
    c->grid_ptrs.assign(n_solids, grid);
    Plan p;
    if ((rc = plan_call(c, c->grid_ptrs.data(), sol.data(), n_solids, opt, nullptr, &p)) !=
        RMX_OK)
        return rc;
    if ((rc = ensure_ws(c, p.ws_bytes)) != RMX_OK) return rc;
    // Step workspace: the step descriptors and the two list lengths (uploaded, the lengths
    // as 0), then 30 doubles per box cell: per axis the transverse advecting velocity and
    // the three chosen transverse xi states (12), and the expansions of the three xi
    // components to the cell's +a and -a faces (18); then the two row-segment lists.
    if (p.total_words >= (int64_t)0x7fffffff) return RMX_E_BOX;
    const size_t ncount = 2 * kStepLists;
    const size_t up = sizeof(StepDev) * n_solids + ncount * sizeof(int32_t);
    const size_t desc = (up + 255) & ~size_t(255);
    const size_t fields = sizeof(double) * 30 * (size_t)p.total_cells;
    const int64_t cap = step_list_cap(p.total_words);
    const size_t need = desc + fields + ncount * sizeof(int32_t) * (size_t)cap;
    if (need > c->step_ws_size) {
        if (c->fixed) return RMX_E_WORKSPACE;
        if (c->step_ws) {
            if (hipDeviceSynchronize() != hipSuccess) return RMX_E_HIP;
            (void)hipFree(c->step_ws);
            c->step_ws = nullptr;
            c->step_ws_size = 0;
        }
        if (hipMalloc(&c->step_ws, need) != hipSuccess) {
            c->step_ws = nullptr;
            return RMX_E_HIP;
        }
        c->step_ws_size = need;
    }
    std::vector<StepDev> sd(n_solids);
    double* trans = reinterpret_cast<double*>(static_cast<char*>(c->step_ws) + desc);
    for (int i = 0; i < n_solids; ++i) {
        const rmx_step_solid& t = ss[i];
        sd[i].xi_n = t.xi_n;
        sd[i].labels_n = t.labels_n;
        sd[i].u = t.u;
        for (int a = 0; a < 3; ++a) sd[i].uf[a] = t.uf[a];
        sd[i].xi_half = t.xi_half;
        sd[i].trans = trans;
        sd[i].faces = trans + 12 * p.solids[i].ncell;
        trans += 30 * p.solids[i].ncell;
    }
    Staging* sg = nullptr;
    if ((rc = get_stage(c, up, &sg)) != RMX_OK) return rc;
    std::memcpy(sg->host, sd.data(), sizeof(StepDev) * n_solids);
    std::memset(static_cast<char*>(sg->host) + sizeof(StepDev) * n_solids, 0,
                ncount * sizeof(int32_t));
    if (hipMemcpyAsync(c->step_ws, sg->host, up, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(sg->ev, st) != hipSuccess)
        return RMX_E_HIP;
    sg->pending = true;
    char* wsb = static_cast<char*>(c->step_ws);
    StepBatch sb{};
    sb.steps = reinterpret_cast<const StepDev*>(wsb);
    sb.counts = reinterpret_cast<int32_t*>(wsb + sizeof(StepDev) * n_solids);
    sb.lists = reinterpret_cast<int32_t*>(wsb + desc + fields);
    sb.list_cap = cap;
    for (int a = 0; a < 3; ++a) {
        sb.lam[a] = dt / (grid->spacing[a] > 0.0 ? grid->spacing[a] : grid->h);
        sb.hl[a] = 0.5 * sb.lam[a];
    }
    rc = launch_planned(c, p, n_solids, opt, st, false, 0, sync, c->ws, c->ws_size, false, &sb);
    if (rc != RMX_OK) return rc;
    if (!sync) return RMX_OK;
    return finish_sync(c, st, n_solids, stats);
}

// Blur-zone consumers: the solid table and the per-tile candidate lists (boxes dilated by
// one cell, so that a face sees the solids of its low cell), uploaded to the context's
// blur workspace on `st`.
static int blur_setup(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids, int32_t n,
                      double eps, const double* G, double* const* phi, bool stress,
                      hipStream_t st, BlurBatch* b) {
    if (!c || !grid || !solids || n < 1) return RMX_E_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps)) return RMX_E_ARG;
    int rc;
    for (int i = 0; i < n; ++i) {
        if ((rc = validate_solid(grid, solids + i)) != RMX_OK) return rc;
        if (G && !std::isfinite(G[i])) return RMX_E_ARG;
    }
    const int64_t TS[3] = {kBlurTX, kBlurTY, kBlurTZ};
    int64_t T[3], nt = 1;
    for (int a = 0; a < 3; ++a) {
        T[a] = (grid->n[a] + TS[a] - 1) / TS[a];
        nt *= T[a];
    }
    if (nt > (int64_t)1 << 30) return RMX_E_ARG;
    std::vector<int32_t> count(nt + 1, 0);
    // The tiles along axis a that the solid's box, dilated by one cell, touches: one run
    // on a walled axis; on a periodic one the cells wrap, and each tile is listed once.
    auto axis_tiles = [&](const rmx_solid& s, int a, std::vector<int64_t>* out) {
        out->clear();
        const int64_t n = grid->n[a];
        if (!grid->periodic[a]) {
            const int64_t lo = std::max<int64_t>(s.lo[a] - 1, 0);
            const int64_t hi = std::min<int64_t>(s.lo[a] + s.ext[a] + 1, n);   // excl.
            for (int64_t t = lo / TS[a]; t <= (hi - 1) / TS[a]; ++t) out->push_back(t);
            return;
        }
        std::vector<char> hit(T[a], 0);
        const int64_t span = std::min<int64_t>(s.ext[a] + 2, n);
        for (int64_t q = 0; q < span; ++q) hit[((s.lo[a] - 1 + q + n) % n) / TS[a]] = 1;
        for (int64_t t = 0; t < T[a]; ++t)
            if (hit[t]) out->push_back(t);
    };
    std::vector<int64_t> ax[3];
    for (int m = 0; m < n; ++m) {
        for (int a = 0; a < 3; ++a) axis_tiles(solids[m], a, &ax[a]);
        for (int64_t z : ax[2])
            for (int64_t y : ax[1])
                for (int64_t x : ax[0]) ++count[(z * T[1] + y) * T[0] + x + 1];
    }
    for (int64_t t = 0; t < nt; ++t) count[t + 1] += count[t];
    std::vector<int32_t> list(count[nt]), fill(count.begin(), count.end() - 1), active;
    for (int m = 0; m < n; ++m) {   // ascending solid index in every tile
        for (int a = 0; a < 3; ++a) axis_tiles(solids[m], a, &ax[a]);
        for (int64_t z : ax[2])
            for (int64_t y : ax[1])
                for (int64_t x : ax[0]) list[fill[(z * T[1] + y) * T[0] + x]++] = m;
    }
    for (int64_t t = 0; t < nt; ++t)
        if (count[t + 1] > count[t]) active.push_back((int32_t)t);
    std::vector<BlurDev> sd(n);
    for (int m = 0; m < n; ++m) {
        const rmx_solid& s = solids[m];
        BlurDev& d = sd[m];
        d = BlurDev{};
        for (int a = 0; a < 3; ++a) {
            d.lo[a] = s.lo[a];
            d.ext[a] = s.ext[a];
            d.centre[a] = s.phi0.centre[a];
        }
        d.L = s.n_layers;
        d.kind = s.phi0.kind;
        if (s.phi0.kind == RMX_SPHERE) {
            d.semi[0] = d.semi[1] = d.semi[2] = s.phi0.semi_axes[0];
            for (int q = 0; q < 9; ++q) d.rot[q] = (q % 4 == 0) ? 1.0 : 0.0;
        } else {
            for (int a = 0; a < 3; ++a) d.semi[a] = s.phi0.semi_axes[a];
            for (int q = 0; q < 9; ++q) d.rot[q] = s.phi0.rot[q];
        }
        d.xi = s.xi;
        d.labels = s.labels;
        d.phi = phi ? phi[m] : nullptr;
        d.G = G ? G[m] : 0.0;
    }
    // the fill's rows along x: per solid its box's cells (H), or per axis a and component
    // the box's faces along a (ext_a + 1 of them, at most n on a periodic axis)
    int64_t rows = 0;
    for (int m = 0; m < n; ++m) {
        sd[m].row0 = rows;
        const rmx_solid& s = solids[m];
        if (!stress) {
            rows += (int64_t)s.ext[1] * s.ext[2];
            continue;
        }
        for (int a = 0; a < 3; ++a) {
            int64_t e[3];
            for (int x = 0; x < 3; ++x) {
                e[x] = s.ext[x] + (x == a ? 1 : 0);
                if (grid->periodic[x] && e[x] > grid->n[x]) e[x] = grid->n[x];
            }
            rows += 6 * e[1] * e[2];
        }
    }
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t o_start = al(sizeof(BlurDev) * n);
    const size_t o_list = o_start + al(sizeof(int32_t) * (nt + 1));
    const size_t o_active = o_list + al(sizeof(int32_t) * std::max<size_t>(list.size(), 1));
    // the scan's count of covered tiles (uploaded as 0) and their list
    const size_t o_ncov = o_active + al(sizeof(int32_t) * std::max<size_t>(active.size(), 1));
    const size_t o_cov = o_ncov + 256;
    const size_t up = o_ncov + sizeof(int32_t);   // bytes uploaded
    const size_t bytes = o_cov + sizeof(int32_t) * std::max<size_t>(active.size(), 1);
    if (hipSetDevice(c->device) != hipSuccess) return RMX_E_HIP;
    if (bytes > c->blur_ws_size) {
        if (c->fixed) return RMX_E_WORKSPACE;
        if (c->blur_ws) {
            if (hipDeviceSynchronize() != hipSuccess) return RMX_E_HIP;
            (void)hipFree(c->blur_ws);
            c->blur_ws = nullptr;
            c->blur_ws_size = 0;
        }
        if (hipMalloc(&c->blur_ws, bytes) != hipSuccess) {
            c->blur_ws = nullptr;
            return RMX_E_HIP;
        }
        c->blur_ws_size = bytes;
    }
    Staging* sg = nullptr;
    if ((rc = get_stage(c, up, &sg)) != RMX_OK) return rc;
    char* h = static_cast<char*>(sg->host);
    std::memcpy(h, sd.data(), sizeof(BlurDev) * n);
    std::memcpy(h + o_start, count.data(), sizeof(int32_t) * (nt + 1));
    if (!list.empty()) std::memcpy(h + o_list, list.data(), sizeof(int32_t) * list.size());
    if (!active.empty()) std::memcpy(h + o_active, active.data(), sizeof(int32_t) * active.size());
    const int32_t zero = 0;
    std::memcpy(h + o_ncov, &zero, sizeof(zero));
    if (hipMemcpyAsync(c->blur_ws, h, up, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(sg->ev, st) != hipSuccess)
        return RMX_E_HIP;
    sg->pending = true;
    char* base = static_cast<char*>(c->blur_ws);
    *b = BlurBatch{};
    b->solids = reinterpret_cast<const BlurDev*>(base);
    b->n_solids = n;
    b->spheres = 1;
    for (int i = 0; i < n; ++i) b->spheres &= solids[i].phi0.kind == RMX_SPHERE ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        b->grid[a] = grid->n[a];
        b->periodic[a] = grid->periodic[a] ? 1 : 0;
        b->tiles[a] = (int32_t)T[a];
        b->h[a] = grid->spacing[a] > 0.0 ? grid->spacing[a] : grid->h;
    }
    b->n_active = (int32_t)active.size();
    b->tile_start = reinterpret_cast<const int32_t*>(base + o_start);
    b->tile_list = reinterpret_cast<const int32_t*>(base + o_list);
    b->active = reinterpret_cast<const int32_t*>(base + o_active);
    b->n_covered = reinterpret_cast<int32_t*>(base + o_ncov);
    b->covered = reinterpret_cast<int32_t*>(base + o_cov);
    b->eps = eps;
    b->fill_rows = rows;
    return RMX_OK;
}

int rmx_blur(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
             double eps, double* H, double* const* phi, void* hip_stream) {
    if (!H && !phi) return RMX_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    BlurBatch b;
    int rc = blur_setup(c, grid, solids, n_solids, eps, nullptr, phi, false, st, &b);
    if (rc != RMX_OK) return rc;
    b.H = H;
    return launch_blur_heaviside(b, st) == hipSuccess ? RMX_OK : RMX_E_HIP;
}

int rmx_solid_stress(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids,
                     int32_t n_solids, double eps, const double* G, double* const* tau,
                     void* hip_stream) {
    if (!G || !tau || !tau[0] || !tau[1] || !tau[2]) return RMX_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    BlurBatch b;
    int rc = blur_setup(c, grid, solids, n_solids, eps, G, nullptr, true, st, &b);
    if (rc != RMX_OK) return rc;
    for (int a = 0; a < 3; ++a) b.tau[a] = tau[a];
    return launch_blur_stress(b, st) == hipSuccess ? RMX_OK : RMX_E_HIP;
}

int rmx_layers_for_blur(double eps, double h, double stretch, int32_t reach, uint32_t flags,
                        int32_t* L) {
    if (!L || !(eps > 0.0) || !(h > 0.0) || !(stretch >= 1.0) || !std::isfinite(eps) ||
        !std::isfinite(h) || !std::isfinite(stretch) || reach < 0)
        return RMX_E_ARG;
    const double D = stretch * eps + std::sqrt(3.0) * h;
    const double cells = (flags & RMX_FLAG_ADJ26) ? D / h : std::sqrt(3.0) * D / h;
    const double l = std::ceil(cells) + (double)reach;
    if (!(l <= RMX_MAX_LAYERS)) return RMX_E_LAYERS;
    *L = (int32_t)l;
    return RMX_OK;
}

int rmx_layers_for_blur_grid(const rmx_grid* grid, double eps, double stretch, int32_t reach,
                             uint32_t flags, int32_t* L) {
    if (!grid || !L || !(grid->h > 0.0) || !std::isfinite(grid->h) || !(eps > 0.0) ||
        !std::isfinite(eps) || !(stretch >= 1.0) || !std::isfinite(stretch) || reach < 0)
        return RMX_E_ARG;
    double d2 = 0.0, inv2 = 0.0, dmin = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!(grid->spacing[a] >= 0.0) || !std::isfinite(grid->spacing[a])) return RMX_E_ARG;
        const double d = grid->spacing[a] > 0.0 ? grid->spacing[a] : grid->h;
        d2 += d * d;
        inv2 += 1.0 / (d * d);
        dmin = a == 0 ? d : std::min(dmin, d);
    }
    const double D = stretch * eps + std::sqrt(d2);
    const double cells = (flags & RMX_FLAG_ADJ26) ? D / dmin : D * std::sqrt(inv2);
    const double l = std::ceil(cells) + (double)reach;
    if (!(l <= RMX_MAX_LAYERS)) return RMX_E_LAYERS;
    *L = (int32_t)l;
    return RMX_OK;
}

int rmx_extrapolate_noalloc(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids,
                            int32_t n_solids, const rmx_options* opt, void* hip_stream,
                            rmx_solid_stats* stats) {
    if (!c || !grid || !solids || n_solids < 1) return RMX_E_ARG;
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    int rc = validate_options(opt);
    if (rc != RMX_OK) return rc;
    for (int i = 0; i < n_solids; ++i)
        if ((rc = validate_solid(grid, solids + i)) != RMX_OK) return rc;
    // graph capture by the library and profiling events would allocate
    if (opt->flags & (RMX_FLAG_GRAPH | RMX_FLAG_PROFILE)) return RMX_E_ARG;
    if (!c->scratch) return RMX_E_HIP;
    const bool sync = stats || (opt->flags & RMX_FLAG_SYNC);
    if (sync && c->stats_host_n < (size_t)kStatWords * n_solids) return RMX_E_WORKSPACE;
    if (hipSetDevice(c->device) != hipSuccess) return RMX_E_HIP;
    // Plan every launch first: nothing is enqueued unless all of them fit the scratch
    // array and the staging slots.
    const bool per_solid = (opt->flags & RMX_FLAG_PER_SOLID) != 0;
    const int calls = per_solid ? n_solids : 1;
    c->grid_ptrs.assign(n_solids, grid);
    c->noalloc_plans.resize(calls);
    for (int i = 0; i < calls; ++i) {
        Plan& p = c->noalloc_plans[i];
        rc = plan_call(c, c->grid_ptrs.data() + (per_solid ? i : 0), solids + (per_solid ? i : 0),
                       per_solid ? 1 : n_solids, opt, nullptr, &p);
        if (rc != RMX_OK) return rc;
        if (p.ws_bytes > kScratchBytes || p.desc_bytes > kStageBytes) return RMX_E_WORKSPACE;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    for (int i = 0; i < calls; ++i) {
        rc = launch_planned(c, c->noalloc_plans[i], per_solid ? 1 : n_solids, opt, st, false,
                            (size_t)kStatWords * (per_solid ? i : 0), sync, c->scratch,
                            kScratchBytes, true);
        if (rc != RMX_OK) return rc;
    }
    if (!sync) return RMX_OK;
    return finish_sync(c, st, n_solids, stats);
}

int rmx_autotune(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
                 const rmx_options* opt, void* hip_stream, int32_t reps, rmx_tuning* best) {
    if (!c || !grid || !solids || n_solids < 1 || !best || reps < 1) return RMX_E_ARG;
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    int rc = validate_options(opt);
    if (rc != RMX_OK) return rc;
    for (int i = 0; i < n_solids; ++i)
        if ((rc = validate_solid(grid, solids + i)) != RMX_OK) return rc;
    if (hipSetDevice(c->device) != hipSuccess) return RMX_E_HIP;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    rmx_options o = *opt;
    o.flags &= ~(uint32_t)(RMX_FLAG_GRAPH | RMX_FLAG_PROFILE | RMX_FLAG_SYNC | RMX_FLAG_PER_SOLID);
    c->grid_ptrs.assign(n_solids, grid);
    Plan probe;
    rc = plan(c->grid_ptrs.data(), solids, n_solids, &o, c->lds_limit, c->cus, Tuning{}, &probe);
    if (rc != RMX_OK) return rc;
    int Wmax = 1;
    for (const auto& d : probe.solids) Wmax = std::max(Wmax, d.W);
    // save xi
    std::vector<size_t> bytes(n_solids), off(n_solids);
    size_t total = 0;
    for (int i = 0; i < n_solids; ++i) {
        bytes[i] = 24 * (size_t)solids[i].ext[0] * solids[i].ext[1] * solids[i].ext[2];
        off[i] = total;
        total += bytes[i];
    }
    char* save = nullptr;
    if (hipStreamSynchronize(st) != hipSuccess) return RMX_E_HIP;
    if (hipMalloc(&save, total) != hipSuccess) return RMX_E_HIP;
    auto copy = [&](bool restore) -> hipError_t {
        for (int i = 0; i < n_solids; ++i) {
            void* a = save + off[i];
            void* x = solids[i].xi;
            const hipError_t e = restore ? hipMemcpyAsync(x, a, bytes[i], hipMemcpyDeviceToDevice, st)
                                         : hipMemcpyAsync(a, x, bytes[i], hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = RMX_OK;
    if (copy(false) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        rc = RMX_E_HIP;
    Tuning win{};
    double win_ms = 1e300;
    const int tws[3] = {1, 2, 4};
    const int per_cu[4] = {2, 3, 4, 6};
    for (int a = 0; a < 3 && rc == RMX_OK; ++a) {
        if (tws[a] > 1 && tws[a] > Wmax + 1) continue;           // wider than every row
        if (label_lds_bytes(probe.Lmax, tws[a], Wmax) > c->lds_limit) continue;
        for (int q = 0; q < 4 && rc == RMX_OK; ++q) {
            Tuning t{tws[a], per_cu[q] * c->cus};
            if (copy(true) != hipSuccess) { rc = RMX_E_HIP; break; }
            // one untimed call (workspace growth, descriptor upload), then `reps` timed
            if ((rc = run_batch(c, c->grid_ptrs.data(), solids, n_solids, &o, st, false, 0, false,
                                &t)) != RMX_OK)
                break;
            if (copy(true) != hipSuccess || hipEventRecord(e0, st) != hipSuccess) {
                rc = RMX_E_HIP;
                break;
            }
            for (int r = 0; r < reps && rc == RMX_OK; ++r)
                rc = run_batch(c, c->grid_ptrs.data(), solids, n_solids, &o, st, false, 0, false,
                               &t);
            if (rc != RMX_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = RMX_E_HIP;
                break;
            }
            // (the restore copy before each timed run is outside the events)
            const double per = ms / reps;
            if (per < win_ms) {
                win_ms = per;
                win = t;
            }
        }
    }
    if (rc == RMX_OK && copy(true) != hipSuccess) rc = RMX_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess && rc == RMX_OK) rc = RMX_E_HIP;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(save);
    if (rc != RMX_OK) return rc;
    if (!(win.tile_w > 0)) return RMX_E_ARG;
    c->tuned[tune_key(probe)] = win;
    best->tile_w = win.tile_w;
    best->extrap_blocks = win.extrap_blocks;
    best->ms = win_ms;
    return RMX_OK;
}

int rmx_set_tuning(rmx_ctx* c, const rmx_grid* grid, const rmx_solid* solids,
                   int32_t n_solids, const rmx_options* opt, const rmx_tuning* t) {
    if (!c || !grid || !solids || n_solids < 1 || !t) return RMX_E_ARG;
    if (t->tile_w != 1 && t->tile_w != 2 && t->tile_w != 4) return RMX_E_ARG;
    if (t->extrap_blocks < 1) return RMX_E_ARG;
    rmx_options def;
    rmx_default_options(&def);
    if (!opt) opt = &def;
    int rc = validate_options(opt);
    if (rc != RMX_OK) return rc;
    for (int i = 0; i < n_solids; ++i)
        if ((rc = validate_solid(grid, solids + i, false)) != RMX_OK) return rc;
    c->grid_ptrs.assign(n_solids, grid);
    Plan probe;
    rc = plan(c->grid_ptrs.data(), solids, n_solids, opt, c->lds_limit, c->cus, Tuning{}, &probe);
    if (rc != RMX_OK) return rc;
    int Wmax = 1;
    for (const auto& d : probe.solids) Wmax = std::max(Wmax, d.W);
    if (label_lds_bytes(probe.Lmax, t->tile_w, Wmax) > c->lds_limit) return RMX_E_ARG;
    c->tuned[tune_key(probe)] = Tuning{t->tile_w, t->extrap_blocks};
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
