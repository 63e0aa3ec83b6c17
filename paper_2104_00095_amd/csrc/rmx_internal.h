// Internal layout shared by the host core and the HIP kernels of librmx.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmx {

constexpr int kMaxLayers = 16;
constexpr int kMaxRadius = 4;
constexpr int kLT = kMaxLayers + 1;          // per-tile layer table stride
constexpr int kTileJ = 16;                   // rows of a label tile along y
constexpr int kTileK = 16;                   // rows of a label tile along z
constexpr int kChunkWords = 64;              // mask words per classification chunk
constexpr int kLocateChunk = 64;             // band indices per chunk_tile entry

// Per-solid device statistics (int64 words).
constexpr int kStatWords = 24;
constexpr int ST_INTERIOR = 0;  // 1..16: band cells of layer l
constexpr int ST_GROWN = 17;
constexpr int ST_NONORMAL = 18;
constexpr int ST_F1 = 19;
constexpr int ST_F2 = 20;
constexpr int ST_FLAGS = 21;
constexpr unsigned long long FLAG_TRUNCATED = 1ull;

constexpr int kDecF1 = 32;
constexpr int kDecF2 = 33;
constexpr int kDecNoNormal = 64;

// One solid as the kernels see it.
struct DevSolid {
    int32_t n0, n1, n2;      // box extents (x fastest)
    int32_t W;               // 64-cell mask words per row
    int32_t ty, tz;          // label tiles along y and z
    int32_t L;               // layers
    int32_t kind;            // 1 sphere, 2 ellipsoid
    int32_t wall_lo[3];      // 1 if the low face along the axis is a grid wall
    int32_t wall_hi[3];
    int32_t tile_base;       // first global tile index of the solid
    int32_t n_tiles;         // tiles of the solid
    int32_t ntx;             // tiles along x (tile_w words each)
    int32_t chunk_base;      // first classification chunk of the solid
    // fused path: z-slabs of kTileK planes, 8^3 bricks, counters and brick lists
    int32_t n_slabs;
    int32_t nbx, nby;        // bricks along x, y
    int32_t bcap;            // brick capacity of one slab: nbx * nby * 2
    int32_t parts;           // extrapolation items per (slab, layer)
    int32_t has_nonwall;     // some box face is not a grid wall (truncation possible)
    int32_t total_chunks;    // classification items of the solid
    int32_t ctr;             // first counter of the solid
    int32_t pad0;
    int64_t list;            // first brick-list entry of the solid
    int64_t ncell;
    int64_t word_base;       // first global mask word
    int64_t slot_base;       // first slot in the slot buffer
    double centre[3];
    double semi[3];
    double rot[9];
    double* xi;
    const double* xi_normal; // field the normals come from (xi if none given)
    double* normals;         // fused path: [3][ncell] normals of the band cells, or null
    int8_t* labels;
    int8_t* decisions;       // nullable
    unsigned long long* mask;  // [n2 * n1][W]
};

// Device tables of one batched call (all in the workspace).
struct Batch {
    const DevSolid* solids;
    int32_t n_solids;
    int32_t n_tiles;
    int32_t Lmax;
    int32_t normal_layers;
    int32_t r_s, r_max;
    int32_t tile_w;          // 64-cell words per label tile along x (1..4)
    int32_t tile_cells;      // slot capacity of a tile: 64 * tile_w * 16 * 16
    int64_t total_words;
    int32_t n_chunks;        // classification chunks (kChunkWords mask words each)
    int32_t chunk_cap;       // entries per layer of chunk_tile
    int64_t slot_cap;        // slot capacity (n_tiles * kTileCells)
    const int32_t* tile_solid;  // [n_tiles]
    int32_t* tile_cnt;       // [n_tiles][kLT] cells of layer l (0: interior) in the tile
    int32_t* tile_lstart;    // [n_tiles][kLT] first slot of layer l within the tile
    int32_t* tile_off;       // [kLT][n_tiles + 1] exclusive prefix over tiles, per layer
    int32_t* chunk_tile;     // [kLT][chunk_cap] tile holding band index 64c of layer l
    int32_t* chunk_flag;     // [n_chunks] 1 if the chunk found a truncating interior cell
    int32_t* slots;          // [slot_cap] linear cell index within the solid's box
    double* normals;         // [3][slot_cap] unnormalised gradient of phi0(xi)
    unsigned long long* stats;  // [n_solids][kStatWords]
};

// Fused persistent path: one launch, work items taken by ticket in an order where every
// dependency precedes its dependents.
enum : uint8_t { FI_CLASSIFY = 0, FI_LABEL = 1, FI_EXTRAP = 2 };
struct FItem {
    uint8_t type;
    uint8_t layer;
    uint16_t slab;
    uint16_t solid;
    uint16_t idx;            // chunk / tile within the slab, or extrapolation part
};
constexpr int kBrick = 8;                    // brick edge (cells)
constexpr int kBrickHalo = 2;                // r_s of the paper
constexpr int kBrickSpan = kBrick + 2 * kBrickHalo;   // 12
constexpr int kBrickCells = kBrickSpan * kBrickSpan * kBrickSpan;  // 1728
constexpr size_t kBrickLds = kBrickCells * 25 + 512 * 2;   // xi + labels + cell list
// counters: [0] ticket, [1] finished blocks, [2] error; per solid from its `ctr`:
// +0 classified chunks, +1 truncated, +2 radius grown, +3 no normal, +4 F1, +5 F2, then
// per slab: classified chunks, labelled tiles; per (layer, slab): finished extrapolation
// items, bricks listed.
constexpr int kCtrGlobal = 4;
constexpr int kCtrSolid = 6;
constexpr unsigned long long FLAG_TIMEOUT = 2ull;

struct Fused {
    const FItem* items;
    int32_t n_items;
    int32_t ctr_words;       // counters used by this call (reset at the end)
    int* ctr;
    int32_t* lists;
    int32_t lds_work;        // bytes of the item work area at the start of the dynamic LDS
    int32_t pad0;
};
// block state after the work area: scan slots, ticket, last flag; brick flags
constexpr int kFusedSmallInts = 8;
constexpr size_t kFusedSmallBytes = kFusedSmallInts * sizeof(int) + kMaxLayers * 32;

// Launchers (rmx_kernels.hip, rmx_fused.hip).
hipError_t launch_classify(const Batch& b, hipStream_t st);
size_t label_lds_bytes(int Lmax, int tile_w, int Wmax);
hipError_t launch_label(const Batch& b, size_t lds, hipStream_t st);
hipError_t launch_scan(const Batch& b, hipStream_t st);
hipError_t launch_normal(const Batch& b, int64_t max_cells, hipStream_t st);
hipError_t launch_extrap(const Batch& b, int layer, int precision, int64_t max_cells,
                         hipStream_t st);
size_t fused_lds_bytes(size_t label_lds);
hipError_t fused_grid(int precision, size_t lds, int device, int* blocks);
hipError_t launch_fused(const Batch& b, const Fused& f, int precision, size_t lds, int blocks,
                        hipStream_t st);

}  // namespace rmx
