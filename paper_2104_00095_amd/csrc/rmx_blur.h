// Device tables and launchers of the blur-zone consumers of the extrapolated reference
// maps (Lin, Derr & Rycroft, arXiv 2104.00095: "Blurred interface method and monolithic
// governing equations", eq. (sm_heavi); SI "Stress calculations", eq. (mod_heaviside)).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rmx {

// Tiles of 8^3 grid cells (two per thread).  (64 x 4 x 2 tiles, whose waves write whole
// 512-byte rows, measured no faster on cavity256 and twice as slow on the suspension: a
// wider tile lists more candidate solids for every cell.)
constexpr int kBlurTX = 8, kBlurTY = 8, kBlurTZ = 8;
constexpr int kBlurTileCells = kBlurTX * kBlurTY * kBlurTZ;

// One solid: its box in the grid, phi0, and its fields (from an extrapolation call).
struct BlurDev {
    int32_t lo[3], ext[3];
    int32_t L, kind;
    double centre[3], semi[3], rot[9];   // a sphere: semi = R (three times), rot = I
    const double* xi;                    // [3][e2][e1][e0]
    const int8_t* labels;                // [e2][e1][e0]
    double* phi;                         // [e2][e1][e0] or null
    double G;                            // shear modulus
    int64_t row0;                        // first row of the solid in the fill's rows
};

struct BlurBatch {
    const BlurDev* solids;
    int32_t n_solids;
    int32_t grid[3];
    int32_t periodic[3];         // 1: the grid wraps along the axis (n faces, not n + 1)
    int32_t tiles[3];            // tiles along x, y, z
    int32_t n_active;
    int32_t spheres;             // every solid is a sphere: the full kernels' sphere-only form
    const int32_t* tile_start;   // [tiles + 1]: candidate solids of each tile (CSR)
    const int32_t* tile_list;    // ascending solid indices (boxes dilated by one cell)
    const int32_t* active;       // tiles with a candidate
    int32_t* n_covered;          // tiles of `active` with a covered cell (zeroed per call)
    int32_t* covered;            // [n_active]: those tiles, in the order the scan found them
    int64_t fill_rows;           // rows (along x) of the boxes' cells or faces, all solids
    double eps;
    double h[3];                 // spacing of each axis
    double* H;                   // [n2][n1][n0] or null
    double* tau[3];              // [6][n2 + f2][n1 + f1][n0 + f0] or null, f_b = 1 if b == a
                                 // and axis a is walled, else 0
};

hipError_t launch_blur_heaviside(const BlurBatch& b, hipStream_t st);
hipError_t launch_blur_stress(const BlurBatch& b, hipStream_t st);

}  // namespace rmx
