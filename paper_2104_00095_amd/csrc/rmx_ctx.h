// The context object behind rmx_ctx* (host state of one device's calls).
#pragma once
#include <hip/hip_runtime.h>

#include <unordered_map>
#include <vector>

#include "rmx.h"
#include "rmx_core.h"
#include "rmx_step.h"

namespace rmx {

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

}  // namespace rmx

struct rmx_ctx {
    int device = 0;
    size_t lds_limit = 65536;
    int cus = 256;
    int normal_per_cu = 4;   // resident blocks of the normal kernel per compute unit
    int normal_sphere_per_cu = 4;   // the same, in its sphere-only form
    int band_per_cu[2] = {2, 2};   // ... of the band kernel, FP64 and FP32-accumulate
    bool fixed = false;
    bool exact_ws = false;   // grow the workspace to exactly what a call needs (server)
    void* ws = nullptr;
    size_t ws_size = 0;
    static constexpr int kRing = 4;
    rmx::Staging stage[kRing];
    int stage_next = 0;
    // what the workspace's descriptor region holds now
    bool desc_valid = false;
    const void* desc_ws = nullptr;
    uint64_t desc_hash = 0;
    size_t desc_len = 0;
    std::vector<char> desc_host;
    unsigned long long* stats_host = nullptr;   // pinned, kStatWords per solid
    size_t stats_host_n = 0;
    hipStream_t capture_stream = nullptr;
    std::unordered_map<uint64_t, rmx::GraphEntry> graphs;
    std::unordered_map<uint64_t, rmx::Tuning> tuned;   // launch shapes per tune_key
    std::vector<rmx_solid_stats> tmp_stats;
    std::vector<const rmx_grid*> grid_ptrs;
    void* step_ws = nullptr;   // time step: step descriptors + transverse face states
    size_t step_ws_size = 0;
    void* blur_ws = nullptr;   // blur-zone consumers: solid table and tile lists
    size_t blur_ws_size = 0;
    void* scratch = nullptr;   // device address of this device's allocation-free workspace
    std::vector<rmx::Plan> noalloc_plans;
    rmx::Profiler prof;
};

namespace rmx {

// Pinned host statistics of at least n words.
int ctx_stats_host(rmx_ctx* c, size_t n);
// Shape class of a planned call (the key of the tuned launch shapes).
uint64_t tune_key(const Plan& p);
// Plan one batched call: the batch with the tuned launch shapes applied (`force`, if
// given, overrides them).
int plan_call(rmx_ctx* c, const rmx_grid* const* grids, const rmx_solid* solids, int n,
              const rmx_options* opt, const Tuning* force, Plan* p);
// Enqueue a planned call on `st` with its workspace at [ws, ws + ws_size): descriptor
// upload, kernels, optional statistics read-back into stats_host + stats_off.  no_alloc:
// nothing is allocated (a staging buffer too small is RMX_E_WORKSPACE).  step (nullable,
// not with use_graph): a time step -- its predictor writes the interior mask in place of
// the classification, and its corrector follows the layer fits; the step's own fields of
// the batch are step->steps, lam and hl (the rest is filled in here).
int launch_planned(rmx_ctx* c, Plan& p, int n, const rmx_options* opt, hipStream_t st,
                   bool use_graph, size_t stats_off, bool want_stats, void* ws, size_t ws_size,
                   bool no_alloc, const StepBatch* step = nullptr);
// Wait for `st`, convert the statistics of n_solids solids into `stats` (nullable) and
// return the first negative per-solid status, else RMX_OK.
int finish_sync(rmx_ctx* c, hipStream_t st, int n_solids, rmx_solid_stats* stats);
// Enqueue one batched call on `st` in the context's own workspace (grown on demand).
// `force` overrides the tuned launch shapes.
int run_batch(rmx_ctx* c, const rmx_grid* const* grids, const rmx_solid* solids, int n,
              const rmx_options* opt, hipStream_t st, bool use_graph, size_t stats_off,
              bool want_stats, const Tuning* force);

}  // namespace rmx
