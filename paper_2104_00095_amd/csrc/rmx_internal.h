// Internal layout shared by the host core and the HIP kernels of librmx.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmx {

constexpr int kMaxLayers = 16;
constexpr int kMaxRadius = 4;
constexpr int kTileJ = 16;                   // rows of a label tile along y
constexpr int kTileK = 16;                   // rows of a label tile along z
constexpr int kMaxTileW = 4;                 // 64-cell words of a label tile along x
constexpr int kXcds = 8;                     // XCDs (workgroups are dealt round-robin)
constexpr int kChunkWords = 16;              // mask words per classification chunk
constexpr int kLT = kMaxLayers + 1;          // per-tile counts: interior, layers 1..16
// Brick lists are split into buckets (tile t appends to bucket t % kBuckets) so that no
// device-wide counter takes more than a few dozen atomic additions per call.
constexpr int kBuckets = 64;

// Per-solid device statistics (int64 words).
constexpr int kStatWords = 24;
constexpr int ST_INTERIOR = 0;  // 1..16: band cells of layer l
constexpr int ST_GROWN = 17;
constexpr int ST_NONORMAL = 18;
constexpr int ST_F1 = 19;
constexpr int ST_F2 = 20;
constexpr int ST_FLAGS = 21;
constexpr unsigned long long FLAG_TRUNCATED = 1ull;
constexpr unsigned long long FLAG_OVERFLOW = 2ull;   // brick list full (never expected)
constexpr unsigned long long FLAG_TIMEOUT = 4ull;    // a bounded wait of the band launch ran out

constexpr int kDecF1 = 32;
constexpr int kDecF2 = 33;
constexpr int kDecNoNormal = 64;

// Bricks: the extrapolation of one layer stages an 8^3 brick of cells with a halo of
// r_s = 2 (12^3 cells: xi and labels) in LDS and fits the brick's cells of that layer.
constexpr int kBrick = 8;
constexpr int kBrickHalo = 2;
constexpr int kBrickSpan = kBrick + 2 * kBrickHalo;                // 12
constexpr int kBrickCells = kBrickSpan * kBrickSpan * kBrickSpan;  // 1728
// LDS of a brick: staged xi (FP64, or FP32 offsets in the reduced-precision form), one
// state byte per cell, and the list of the brick's layer cells.
constexpr size_t brick_lds_bytes(int precision) {
    return kBrickCells * (3 * (precision == 1 ? 4 : 8) + 1) + 512 * 2;
}

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
    int32_t nbx, nby, nbz;   // 8^3 bricks along x, y, z
    int32_t aniso;           // unequal spacings: the normal factor takes rho into account
    int64_t ncell;
    int64_t word_base;       // first global mask word
    double centre[3];
    double semi[3];
    double rot[9];
    double rho[3];           // spacing of each axis over the smallest (1, 1, 1 when equal)
    double irho[3];          // 1 / rho
    double* xi;
    const double* xi_normal; // field the normals come from (xi if none given)
    double* normals;         // [3][ncell]: unnormalised normals of cells of layers <= nl
    int8_t* labels;
    int8_t* decisions;       // nullable
    unsigned long long* mask;  // [n2 * n1][W]
};

// Control words of the persistent band launch (in the workspace, zeroed by the
// classification of the call).
struct BandCtl {
    int taken[kMaxLayers + 1][kXcds];  // items handed out from each queue of each phase
    int done[kMaxLayers + 1];          // items completed per phase (0: normals, l: layer l)
    int err;                           // a bounded wait ran out
    int pad[14];
};

// Device tables of one batched call (all in the workspace).
struct Batch {
    const DevSolid* solids;
    int32_t n_solids;
    int32_t n_tiles;
    int32_t Lmax;
    int32_t normal_layers;
    int32_t r_s, r_max;
    int32_t tile_w;          // 64-cell words per label tile along x (1..kMaxTileW)
    int32_t n_chunks;        // classification chunks (kChunkWords mask words each)
    int32_t adj26;           // layers by the 26-neighbour adjacency (else face neighbours)
    int32_t spheres;         // every solid of the call is a sphere (the normal kernel's
                             // sphere-only form)
    int64_t total_words;
    int64_t blist_cap;       // brick-list entries per layer: n_tiles * 32 * tile_w
    const int32_t* tile_solid;  // [n_tiles]
    int32_t* tile_cnt;       // [n_tiles][kLT] interior and per-layer cells of each tile
    unsigned long long* stats;  // [n_solids][kStatWords], zeroed by the classification
    int32_t* bcount;         // [kMaxLayers][kBuckets] bricks listed, zeroed likewise
    unsigned long long* blist;  // [Lmax][blist_cap]: solid << 32 | bz << 20 | by << 10 | bx
    int64_t dlist_cap;       // dense brick-list entries per layer: the bricks of all boxes
    int32_t* dcount;         // [kMaxLayers] bricks of each layer, written by the normal kernel
    unsigned long long* dlist;  // [Lmax][dlist_cap]: each layer's bricks, contiguous
    BandCtl* band;           // the persistent band launch's counters
};

// Bucket b of a layer's brick list holds the bricks of tiles t = b (mod kBuckets), at
// most 32 * tile_w per tile; its region starts at bucket_base(b) entries.
__host__ __device__ inline int64_t bucket_base(int b, int n_tiles, int tile_w) {
    const int q = n_tiles / kBuckets, r = n_tiles % kBuckets;
    return (int64_t)32 * tile_w * ((int64_t)b * q + (b < r ? b : r));
}

// Launchers (rmx_kernels.hip).
hipError_t launch_classify(const Batch& b, hipStream_t st);
size_t label_lds_bytes(int Lmax, int tile_w, int Wmax);
hipError_t launch_label(const Batch& b, size_t lds, hipStream_t st);
hipError_t launch_normal(const Batch& b, int blocks, hipStream_t st);
// Blocks of the normal kernel resident per compute unit (occupancy, queried once).
int normal_blocks_per_cu(bool spheres);
hipError_t launch_extrap(const Batch& b, int layer, int precision, int blocks,
                         hipStream_t st);
// The persistent band launch (normals and every layer's fits in one launch).
size_t band_lds_bytes(int precision);
int band_blocks_per_cu(int precision);
hipError_t launch_band(const Batch& b, int precision, int blocks, hipStream_t st);

}  // namespace rmx
