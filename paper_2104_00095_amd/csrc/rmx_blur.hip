// HIP kernels of the blur-zone consumers of the extrapolated reference maps (Lin, Derr &
// Rycroft, arXiv 2104.00095):
//   k_blur_heaviside  per grid cell inside some solid's box: phi_m = phi0_m(xi_m) on the
//                     cells the solid labels 0..L, the smoothed Heaviside of eq. (sm_heavi),
//                     and the multi-body modified Heaviside of eq. (mod_heaviside),
//                     H = max(1 - sum_m (1 - H_eps(phi_m)), 0);
//   k_blur_stress     per cell face with a cell inside some solid's box (SI "Stress
//                     calculations"): for each solid whose difference stencil is labelled,
//                     grad xi by centred differences at the face, F = (grad xi)^{-1},
//                     B = F F^T, tau_m = G_m (B - tr(B)/3 I), the weight 1 - H_eps(phi_m)
//                     at the face's xi; the blend T (sum of weights S <= 1) or T / S.
// A block takes one 8^3 tile of the grid; the solids that can touch it come from a list
// built on the host (boxes dilated by one cell), visited in ascending order, so every sum
// runs in the same order as in any other implementation.  Each consumer runs in three
// launches: a fill writes, row by row along x, the result every cell or face of a box takes
// when no solid covers its stencil (H = 1, zero stress); a scan over every tile with a
// candidate lists the tiles where a candidate labels (0..L) a cell of the tile (dilated by
// one cell for the faces' stencils); the full kernel, whose phi0 and 3x3 inverse hold many
// registers, then computes those tiles only, over the fill's values.  Periodic axes (SI "Test
// cases"): a box holds the solid's unwrapped map and may run past the grid's end; grid
// cell g lies at box coordinate (g - lo) mod n there, and difference stencils are taken in
// box coordinates, so they never join the two ends of a box that spans the axis.  Stencil gathers of FP64 fields
// over the thin blur zones: bandwidth and latency work, no MFMA.
#include "rmx_blur.h"
#include "rmx_device.h"
#include "rmx_weight.h"

namespace rmx {
namespace {
using namespace dev;


__device__ __forceinline__ ShapeR blur_shape(const BlurDev& s) {
    ShapeR r;
    r.kind = s.kind;
    r.c0 = s.centre[0]; r.c1 = s.centre[1]; r.c2 = s.centre[2];
    r.e0 = s.semi[0]; r.e1 = s.semi[1]; r.e2 = s.semi[2];
    r.r00 = s.rot[0]; r.r01 = s.rot[1]; r.r02 = s.rot[2];
    r.r10 = s.rot[3]; r.r11 = s.rot[4]; r.r12 = s.rot[5];
    r.r20 = s.rot[6]; r.r21 = s.rot[7]; r.r22 = s.rot[8];
    return r;
}

// Box coordinates l of grid cell g (0 <= g < n) in the solid's box; false outside it.
__device__ __forceinline__ bool box_coords(const BlurBatch& b, const BlurDev& s, const int g[3],
                                           int l[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int d = g[a] - s.lo[a];
        if (b.periodic[a] && d < 0) d += b.grid[a];   // lo and g lie in [0, n)
        if (d < 0 || d >= s.ext[a]) return false;
        l[a] = d;
    }
    return true;
}

// Index of the cell at box coordinates (x, y, z), or -1 outside the box.
__device__ __forceinline__ int64_t box_cell(const BlurDev& s, int x, int y, int z) {
    if (x < 0 || x >= s.ext[0] || y < 0 || y >= s.ext[1] || z < 0 || z >= s.ext[2])
        return -1;
    return ((int64_t)z * s.ext[1] + y) * s.ext[0] + x;
}

__device__ __forceinline__ bool covered(const BlurDev& s, int64_t c) {
    const int lab = load_global(s.labels + c);
    return lab >= 0 && lab <= s.L;
}

__device__ __forceinline__ void xi_at(const BlurDev& s, int64_t c, double v[3]) {
    const int64_t nc = (int64_t)s.ext[0] * s.ext[1] * s.ext[2];
    v[0] = load_global(s.xi + c);
    v[1] = load_global(s.xi + nc + c);
    v[2] = load_global(s.xi + 2 * nc + c);
}

// The tile of this block and the cell q (0..511) of it in grid coordinates.
__device__ __forceinline__ void tile_cell(const BlurBatch& b, int t, int q, int g[3]) {
    const int tx = t % b.tiles[0], ty = (t / b.tiles[0]) % b.tiles[1];
    const int tz = t / (b.tiles[0] * b.tiles[1]);
    g[0] = tx * kBlurTX + q % kBlurTX;
    g[1] = ty * kBlurTY + (q / kBlurTX) % kBlurTY;
    g[2] = tz * kBlurTZ + q / (kBlurTX * kBlurTY);
}

// ------------------------------------------------------------------------------------
// The scan: does a candidate label any cell of the tile dilated by one cell?  (A face's
// difference stencil reaches one cell beyond its owner's tile; a cell's phi only the cell.)
// ------------------------------------------------------------------------------------
__device__ bool tile_covered(const BlurBatch& b, int t, int e0, int e1, bool dilate) {
    const int tx = t % b.tiles[0], ty = (t / b.tiles[0]) % b.tiles[1];
    const int tz = t / (b.tiles[0] * b.tiles[1]);
    const int h = dilate ? 1 : 0;
    const int o0 = tx * kBlurTX - h, o1 = ty * kBlurTY - h, o2 = tz * kBlurTZ - h;
    const int DX = kBlurTX + 2 * h, DY = kBlurTY + 2 * h, DZ = kBlurTZ + 2 * h;
    int hit = 0;
    for (int e = e0; e < e1; ++e) {
        const BlurDev& s = b.solids[b.tile_list[e]];
        for (int q = threadIdx.x; q < DX * DY * DZ; q += 256) {
            int g[3] = {o0 + q % DX, o1 + (q / DX) % DY, o2 + q / (DX * DY)};
            bool on = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (g[a] >= 0 && g[a] < b.grid[a]) continue;
                if (b.periodic[a])
                    g[a] = g[a] < 0 ? g[a] + b.grid[a] : g[a] - b.grid[a];
                else
                    on = false;
            }
            int l[3];
            if (on && box_coords(b, s, g, l) && covered(s, box_cell(s, l[0], l[1], l[2])))
                hit = 1;
        }
    }
    return __syncthreads_or(hit) != 0;
}

template <bool STRESS>
__global__ __launch_bounds__(256) void k_blur_scan(BlurBatch b) {
    const int t = b.active[blockIdx.x];
    const int e0 = b.tile_start[t], e1 = b.tile_start[t + 1];
    if (tile_covered(b, t, e0, e1, STRESS) && threadIdx.x == 0)
        b.covered[atomicAdd(b.n_covered, 1)] = t;
}

// ------------------------------------------------------------------------------------
// The fill: what a cell or face with no covered stencil takes (H = 1 on a cell inside some
// box; zero stress on a face with a cell inside some box), over every box, one row along x
// per wave (whole cache lines).  Box regions that overlap are written more than once, with
// the same value.  Face rows of axis a span the box's ext_a + 1 faces along a (n on a
// periodic axis that the box spans); rows are ordered per solid, then (for the stress)
// axis, component, z, y.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int fill_extent(const BlurBatch& b, const BlurDev& s, int a, int ax) {
    int e = s.ext[ax] + (ax == a ? 1 : 0);
    if (b.periodic[ax] && e > b.grid[ax]) e = b.grid[ax];
    return e;
}

__device__ __forceinline__ int find_solid_by_row(const BlurBatch& b, int64_t r) {
    int lo = 0, hi = b.n_solids - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.solids[mid].row0 <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// A fill row's place: solid m, axis a and component c (stress only), box row (y, z), and
// the extents E0 x E1 x E2 of the rows' region.
struct FillPos {
    int m, a, c, y, z, E0, E1, E2;
};

template <bool STRESS>
__device__ __forceinline__ void fill_extents(const BlurBatch& b, FillPos& p) {
    const BlurDev& s = b.solids[p.m];
    if (STRESS) {
        p.E0 = fill_extent(b, s, p.a, 0);
        p.E1 = fill_extent(b, s, p.a, 1);
        p.E2 = fill_extent(b, s, p.a, 2);
    } else {
        p.E0 = s.ext[0];
        p.E1 = s.ext[1];
        p.E2 = s.ext[2];
    }
}

// Place of row r (divisions; once per wave).
template <bool STRESS>
__device__ FillPos fill_pos(const BlurBatch& b, int64_t r) {
    FillPos p;
    p.m = uniform_int(find_solid_by_row(b, r));
    int64_t q = r - b.solids[p.m].row0;
    p.a = 0;
    p.c = 0;
    fill_extents<STRESS>(b, p);
    if (STRESS) {
        while (q >= 6 * (int64_t)p.E1 * p.E2) {
            q -= 6 * (int64_t)p.E1 * p.E2;
            ++p.a;
            fill_extents<STRESS>(b, p);
        }
        const int64_t plane = (int64_t)p.E1 * p.E2;
        p.c = (int)(q / plane);
        q -= (int64_t)p.c * plane;
    }
    p.y = (int)(q % p.E1);
    p.z = (int)(q / p.E1);
    return p;
}

// The next row's place (y fastest, then z, component, axis, solid).
template <bool STRESS>
__device__ __forceinline__ void fill_next(const BlurBatch& b, FillPos& p) {
    if (++p.y < p.E1) return;
    p.y = 0;
    if (++p.z < p.E2) return;
    p.z = 0;
    if (STRESS) {
        if (++p.c < 6) return;
        p.c = 0;
        if (++p.a < 3) {
            fill_extents<STRESS>(b, p);
            return;
        }
        p.a = 0;
    }
    if (++p.m < b.n_solids) fill_extents<STRESS>(b, p);
}

// Each wave writes one contiguous run of rows.
template <bool STRESS>
__global__ __launch_bounds__(256) void k_blur_fill(BlurBatch b) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    const int64_t per = (b.fill_rows + waves - 1) / waves;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * per;
    const int64_t r1 = r0 + per < b.fill_rows ? r0 + per : b.fill_rows;
    if (r0 >= r1) return;
    FillPos p = fill_pos<STRESS>(b, r0);
    for (int64_t r = r0; r < r1; ++r, fill_next<STRESS>(b, p)) {
        const BlurDev& s = b.solids[p.m];
        int gy = s.lo[1] + p.y, gz = s.lo[2] + p.z;
        if (b.periodic[1] && gy >= b.grid[1]) gy -= b.grid[1];
        if (b.periodic[2] && gz >= b.grid[2]) gz -= b.grid[2];
        double* out;
        int64_t n0, n1;
        double v;
        if (STRESS) {
            const int a = p.a;
            n0 = b.grid[0] + (a == 0 && !b.periodic[0]);
            n1 = b.grid[1] + (a == 1 && !b.periodic[1]);
            const int64_t n2 = b.grid[2] + (a == 2 && !b.periodic[2]);
            out = b.tau[a] + (int64_t)p.c * (n0 * n1 * n2);
            v = 0.0;
        } else {
            n0 = b.grid[0];
            n1 = b.grid[1];
            out = b.H;
            v = 1.0;
        }
        const int64_t base = ((int64_t)gz * n1 + gy) * n0;
        for (int t = lane; t < p.E0; t += 64) {
            int gx = s.lo[0] + t;
            if (b.periodic[0] && gx >= b.grid[0]) gx -= b.grid[0];
            out[base + gx] = v;
        }
    }
}

// Blocks of the full kernels: they stride over the covered tiles.
constexpr int kBlurFullBlocks = 2048;

// phi0 and the weight 1 - H_eps(phi0), in the sphere-only form (kSpheres: calls whose
// solids are all spheres; the same operations as the general functions' sphere branch,
// without the ellipsoid code and its registers) or the general one.
template <bool kSpheres>
__device__ __forceinline__ double phi0_of(const ShapeR& s, double x0, double x1, double x2) {
    if constexpr (kSpheres)
        return phi0_sphere(s, x0, x1, x2);
    else
        return phi0(s, x0, x1, x2);
}
template <bool kSpheres>
__device__ __forceinline__ double weight_of(const ShapeR& s, double x0, double x1, double x2,
                                            double eps) {
    if constexpr (kSpheres)
        return 1.0 - heaviside_eps(phi0_sphere(s, x0, x1, x2), eps);
    else
        return weight_at(s, x0, x1, x2, eps);
}

// ------------------------------------------------------------------------------------
// Modified Heaviside (and phi_m).
// ------------------------------------------------------------------------------------
template <bool kSpheres>
__device__ void heaviside_tile(const BlurBatch& b, int t) {
    const int e0 = b.tile_start[t], e1 = b.tile_start[t + 1];
    for (int q = threadIdx.x; q < kBlurTileCells; q += 256) {
        int g[3];
        tile_cell(b, t, q, g);
        if (g[0] >= b.grid[0] || g[1] >= b.grid[1] || g[2] >= b.grid[2]) continue;
        bool any = false;
        double acc = 0.0;
        for (int e = e0; e < e1; ++e) {
            const BlurDev& s = b.solids[b.tile_list[e]];
            int l[3];
            if (!box_coords(b, s, g, l)) continue;
            const int64_t c = box_cell(s, l[0], l[1], l[2]);
            any = true;
            if (!covered(s, c)) continue;
            double v[3];
            xi_at(s, c, v);
            if (s.phi) {
                const double p = phi0_of<kSpheres>(blur_shape(s), v[0], v[1], v[2]);
                s.phi[c] = p;
                acc += 1.0 - heaviside_eps(p, b.eps);
            } else {
                acc += weight_of<kSpheres>(blur_shape(s), v[0], v[1], v[2], b.eps);
            }
        }
        if (!any || !b.H) continue;
        const double d = 1.0 - acc;
        b.H[((int64_t)g[2] * b.grid[1] + g[1]) * b.grid[0] + g[0]] = d > 0.0 ? d : 0.0;
    }
}

template <bool kSpheres>
__global__ __launch_bounds__(256) void k_blur_heaviside(BlurBatch b) {
    const int n = *b.n_covered;
    for (int i = blockIdx.x; i < n; i += gridDim.x) heaviside_tile<kSpheres>(b, b.covered[i]);
}

// ------------------------------------------------------------------------------------
// Solid stress at faces.
// ------------------------------------------------------------------------------------
// Neo-Hookean stress of solid s at the face between the cells at box coordinates
// P = f - e_a and Q = f, and its weight; false (no contribution) unless every stencil
// cell lies in the box and is labelled.  h: the spacings.  The axis a is a template
// argument: the Jacobian's columns and the stencil offsets are then fixed at compile time
// and stay in registers.
template <int a, bool kSpheres>
__device__ bool face_stress(const BlurDev& s, const int f[3], const double* h, double eps,
                            double tau[6], double* w) {
    int P[3] = {f[0], f[1], f[2]};
    P[a] -= 1;
    const int64_t cp = box_cell(s, P[0], P[1], P[2]), cq = box_cell(s, f[0], f[1], f[2]);
    if (cp < 0 || cq < 0 || !covered(s, cp) || !covered(s, cq)) return false;
    double xp[3], xq[3];
    xi_at(s, cp, xp);
    xi_at(s, cq, xq);
    double J[3][3];   // J[q][b] = d xi_q / d x_b
#pragma unroll
    for (int q = 0; q < 3; ++q) J[q][a] = (xq[q] - xp[q]) / h[a];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (t == a) continue;
        const int dx = t == 0, dy = t == 1, dz = t == 2;
        const int64_t c1 = box_cell(s, P[0] - dx, P[1] - dy, P[2] - dz);
        const int64_t c2 = box_cell(s, P[0] + dx, P[1] + dy, P[2] + dz);
        const int64_t c3 = box_cell(s, f[0] - dx, f[1] - dy, f[2] - dz);
        const int64_t c4 = box_cell(s, f[0] + dx, f[1] + dy, f[2] + dz);
        if (c1 < 0 || c2 < 0 || c3 < 0 || c4 < 0) return false;
        if (!covered(s, c1) || !covered(s, c2) || !covered(s, c3) || !covered(s, c4))
            return false;
        double v1[3], v2[3], v3[3], v4[3];
        xi_at(s, c1, v1);
        xi_at(s, c2, v2);
        xi_at(s, c3, v3);
        xi_at(s, c4, v4);
#pragma unroll
        for (int q = 0; q < 3; ++q) J[q][t] = ((v2[q] - v1[q]) + (v4[q] - v3[q])) / (4.0 * h[t]);
    }
    // F = J^{-1} by cofactors
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = (J[0][0] * c00 + J[0][1] * c01) + J[0][2] * c02;
    double F[3][3];
    F[0][0] = c00 / det;
    F[1][0] = c01 / det;
    F[2][0] = c02 / det;
    F[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    F[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    F[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    F[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    F[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    F[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double B[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            B[r][c] = (F[r][0] * F[c][0] + F[r][1] * F[c][1]) + F[r][2] * F[c][2];
    const double tr3 = ((B[0][0] + B[1][1]) + B[2][2]) / 3.0;
    const double G = s.G;
    tau[0] = G * (B[0][0] - tr3);
    tau[1] = G * (B[1][1] - tr3);
    tau[2] = G * (B[2][2] - tr3);
    tau[3] = G * B[0][1];
    tau[4] = G * B[0][2];
    tau[5] = G * B[1][2];
    const double x0 = (xp[0] + xq[0]) * 0.5, x1 = (xp[1] + xq[1]) * 0.5,
                 x2 = (xp[2] + xq[2]) * 0.5;
    *w = weight_of<kSpheres>(blur_shape(s), x0, x1, x2, eps);
    return true;
}

// The face f along a (between grid cells f - e_a and f; f[a] in [0, n), or n on a walled
// axis).
template <int a, bool kSpheres>
__device__ void blend_face(const BlurBatch& b, int e0, int e1, const int f[3]) {
    int P[3] = {f[0], f[1], f[2]};
    P[a] -= 1;   // the face's low cell (wrapped on a periodic axis)
    if (b.periodic[a] && P[a] < 0) P[a] += b.grid[a];
    bool any = false;
    double S = 0.0;
    double T[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = e0; e < e1; ++e) {
        const BlurDev& s = b.solids[b.tile_list[e]];
        int lq[3], lp[3];
        const bool inq = f[a] < b.grid[a] && box_coords(b, s, f, lq);
        const bool inp = P[a] >= 0 && box_coords(b, s, P, lp);
        if (!inq && !inp) continue;
        any = true;
        // the face seen from the box: Q's box coordinates, or P's one step up along a
        int q[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) q[c] = inq ? lq[c] : lp[c] + (c == a && !inq);
        double t6[6], w;
        if (!face_stress<a, kSpheres>(s, q, b.h, b.eps, t6, &w)) continue;
        S += w;
#pragma unroll
        for (int c = 0; c < 6; ++c) T[c] += w * t6[c];
    }
    if (!any) return;
    const int64_t n0 = b.grid[0] + (a == 0 && !b.periodic[0]),
                  n1 = b.grid[1] + (a == 1 && !b.periodic[1]),
                  n2 = b.grid[2] + (a == 2 && !b.periodic[2]);
    const int64_t nf = n0 * n1 * n2;
    const int64_t fi = ((int64_t)f[2] * n1 + f[1]) * n0 + f[0];
    double* out = b.tau[a];
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c * nf + fi] = S <= 1.0 ? T[c] : T[c] / S;
}

// A cell's faces along a: its low face, and on a walled axis the last cell's face beyond.
template <int a, bool kSpheres>
__device__ __forceinline__ void cell_faces(const BlurBatch& b, int e0, int e1, const int g[3]) {
    const int nf = (g[a] == b.grid[a] - 1 && !b.periodic[a]) ? 2 : 1;
#pragma unroll 1
    for (int k = 0; k < nf; ++k) {
        int f[3] = {g[0], g[1], g[2]};
        f[a] += k;
        blend_face<a, kSpheres>(b, e0, e1, f);
    }
}

template <bool kSpheres>
__device__ void stress_tile(const BlurBatch& b, int t) {
    const int e0 = b.tile_start[t], e1 = b.tile_start[t + 1];
    for (int q = threadIdx.x; q < kBlurTileCells; q += 256) {
        int g[3];
        tile_cell(b, t, q, g);
        if (g[0] >= b.grid[0] || g[1] >= b.grid[1] || g[2] >= b.grid[2]) continue;
        cell_faces<0, kSpheres>(b, e0, e1, g);
        cell_faces<1, kSpheres>(b, e0, e1, g);
        cell_faces<2, kSpheres>(b, e0, e1, g);
    }
}

// Three waves per SIMD: the face code holds about 190 registers; at 168 a few spill, which
// costs less than the third of the waves it gains on many-body boxes.
template <bool kSpheres>
__global__ __launch_bounds__(256, 3) void k_blur_stress(BlurBatch b) {
    const int n = *b.n_covered;
    for (int i = blockIdx.x; i < n; i += gridDim.x) stress_tile<kSpheres>(b, b.covered[i]);
}

}  // namespace

// Blocks of the fill: four rows per block at a time.
static int fill_grid(const BlurBatch& b) {
    int64_t blocks = (b.fill_rows + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    return (int)(blocks > 0 ? blocks : 1);
}

hipError_t launch_blur_heaviside(const BlurBatch& b, hipStream_t st) {
    if (b.n_active <= 0) return hipSuccess;
    hipError_t e;
    if (b.H) {
        hipLaunchKernelGGL(k_blur_fill<false>, dim3(fill_grid(b)), dim3(256), 0, st, b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_blur_scan<false>, dim3(b.n_active), dim3(256), 0, st, b);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int g = b.n_active < kBlurFullBlocks ? b.n_active : kBlurFullBlocks;
    if (b.spheres)
        hipLaunchKernelGGL(k_blur_heaviside<true>, dim3(g), dim3(256), 0, st, b);
    else
        hipLaunchKernelGGL(k_blur_heaviside<false>, dim3(g), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_blur_stress(const BlurBatch& b, hipStream_t st) {
    if (b.n_active <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_blur_fill<true>, dim3(fill_grid(b)), dim3(256), 0, st, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_blur_scan<true>, dim3(b.n_active), dim3(256), 0, st, b);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int g = b.n_active < kBlurFullBlocks ? b.n_active : kBlurFullBlocks;
    if (b.spheres)
        hipLaunchKernelGGL(k_blur_stress<true>, dim3(g), dim3(256), 0, st, b);
    else
        hipLaunchKernelGGL(k_blur_stress<false>, dim3(g), dim3(256), 0, st, b);
    return hipGetLastError();
}

}  // namespace rmx
