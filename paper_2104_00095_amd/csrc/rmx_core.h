// Host-side planning of one batched call; shared by the context API and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "rmx.h"
#include "rmx_internal.h"

namespace rmx {

struct Plan {
    int n_solids = 0;
    std::vector<DevSolid> solids;
    std::vector<int32_t> tile_solid;
    int n_tiles = 0;
    int n_chunks = 0;
    int chunk_cap = 0;
    int Lmax = 0;
    int normal_layers = 0;
    int tile_w = 1;
    int tile_cells = 0;
    size_t lds_bytes = 0;
    int64_t total_words = 0;
    int64_t slot_cap = 0;
    int64_t total_cells = 0;
    // workspace layout (byte offsets); [0, desc_bytes) is uploaded from the host
    size_t off_desc = 0, off_tile_solid = 0, desc_bytes = 0;
    size_t off_stats = 0, off_tile_cnt = 0, off_tile_lstart = 0, off_tile_off = 0;
    size_t off_chunk_tile = 0, off_chunk_flag = 0;
    size_t off_mask = 0, off_slots = 0, off_normals = 0;
    size_t ws_bytes = 0;
    // fused persistent form
    bool fused = false;
    std::vector<FItem> items;
    int ctr_words = 0;
    size_t off_lists = 0;
};

// Records HIP events around each launch of the chain when attached to rmx_enqueue.
struct Profiler {
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[RMX_N_PHASES] = {};
    int64_t launches[RMX_N_PHASES] = {};
    hipEvent_t get();
    hipError_t begin(int phase, hipStream_t st, Rec* r);
    hipError_t end(Rec& r, hipStream_t st);
    hipError_t drain();
    ~Profiler();
};

}  // namespace rmx

int rmx_validate(const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
                 const rmx_options* opt);
int rmx_plan(const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
             const rmx_options* opt, size_t lds_limit, bool fused, rmx::Plan* p);
void rmx_bind(rmx::Plan* p, void* ws, const rmx_options* opt, rmx::Batch* b);
void rmx_pack_desc(const rmx::Plan& p, void* host);
hipError_t rmx_enqueue(const rmx::Plan& p, const rmx::Batch& b, int precision,
                       hipStream_t st, rmx::Profiler* prof = nullptr);
void rmx_convert_stats(const unsigned long long* dev, int n, rmx_solid_stats* out);
