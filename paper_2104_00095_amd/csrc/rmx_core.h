// Host-side planning and launch sequencing of librmx (shared by the context API and the
// serving loop).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "rmx.h"
#include "rmx_internal.h"

namespace rmx {

// Launch shapes a call may vary without changing any result: the label tile width and
// the number of blocks striding over a layer's brick list.
struct Tuning {
    int tile_w = 0;          // 1, 2 or 4 (0: the widest that fits the LDS)
    int extrap_blocks = 0;   // 0: three per compute unit
};

struct Plan {
    int n_solids = 0;
    std::vector<DevSolid> solids;
    std::vector<int32_t> tile_solid;
    int n_tiles = 0;
    int n_chunks = 0;
    int Lmax = 0;
    int normal_layers = 0;
    int tile_w = 1;
    int extrap_blocks = 1;
    int normal_blocks = 1;
    bool spheres = false;      // every solid is a sphere: the normal kernel's sphere-only form
    bool persistent = false;   // the band work in one persistent launch
    int band_blocks = 1;
    size_t lds_bytes = 0;
    int64_t total_words = 0;
    int64_t total_cells = 0;
    int64_t blist_cap = 0;
    int64_t dlist_cap = 0;
    // workspace layout (byte offsets); [0, desc_bytes) is uploaded from the host
    size_t off_desc = 0, off_tile_solid = 0, desc_bytes = 0;
    size_t off_stats = 0, off_tile_cnt = 0, off_bcount = 0, off_mask = 0, off_normals = 0;
    size_t off_blist = 0, off_dcount = 0, off_dlist = 0, off_band = 0;
    size_t ws_bytes = 0;
    // red zones between regions (CPU emulation build only): (offset, bytes)
    std::vector<std::pair<size_t, size_t>> gaps;
};

#ifdef RMX_EMU_REDZONES
// CPU emulation: make the whole workspace addressable, then poison the red zones.
void rmx_emu_poison_gaps(void* ws, size_t ws_bytes,
                         const std::vector<std::pair<size_t, size_t>>& gaps);
#endif

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

// Validation of one solid against its grid, and of the options.
int validate_options(const rmx_options* opt);
// need_fields = false: the field pointers are not checked (sizing, server templates).
int validate_solid(const rmx_grid* grid, const rmx_solid* s, bool need_fields = true);

// Plan a batch: solid i lives on grid grids[i].  `cu` = compute units of the device,
// `normal_per_cu` = blocks of the normal kernel resident per compute unit, in its general
// and in its sphere-only form.
int plan(const rmx_grid* const* grids, const rmx_solid* solids, int32_t n_solids,
         const rmx_options* opt, size_t lds_limit, int cu, const Tuning& tune, Plan* p,
         int normal_per_cu = 4, int band_per_cu = 2, int normal_sphere_per_cu = 0);
void bind(Plan* p, void* ws, const rmx_options* opt, Batch* b);
void pack_desc(const Plan& p, void* host);
// The launch chain of a planned call.  classify = false: the interior mask is already in
// the workspace (a time step's predictor wrote it), so the chain starts at the labels.
hipError_t enqueue(const Plan& p, const Batch& b, int precision, hipStream_t st,
                   Profiler* prof = nullptr, bool classify = true);
void convert_stats(const unsigned long long* dev, int n, rmx_solid_stats* out);
uint64_t fnv1a(const void* p, size_t n, uint64_t h);

}  // namespace rmx
