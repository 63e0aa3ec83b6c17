// HIP kernels of one time step of the reference map around the extrapolation (Lin, Derr &
// Rycroft, arXiv 2104.00095, SI "Timestepping algorithm", steps 5-7; SI "Evaluating the
// advective term": eq. (adv_terms), the Taylor-expanded face states of xi, the
// Godunov-type upwinding scheme, Colella's fourth-order limited normal slopes, and the
// upwinded tangential derivatives).  A step is
//   k_step_trans    per cell of the old band within reach of the predicted cells, and per
//                   axis t: the transverse face between the cell and its +t neighbour --
//                   the Godunov choice of the advecting t-velocity from its down and up
//                   expansions, and the chosen expansion of each xi component;
//   k_step_faces    per cell next to a predicted cell (labelled 0..L-4 at step n, 3
//                   cells inside the box) and per axis a: the expansions of xi from the
//                   cell to its -a and +a faces with their tangential terms -- each once;
//   k_step_predict  per predicted cell: the Godunov choice of each of its six face states
//                   by the sign of the face velocity, the advective term,
//                   xi^{n+1} = xi^n - dt [(u.grad) xi];
//                   the rest of the old band becomes undefined (NaN); the interior mask
//                   of step n + 1 (predicted cells with phi0(xi^{n+1}) < 0) is written
//                   here, so the extrapolation that follows needs no classification pass;
//   (extrapolation from that mask: labels, normals, layer fits -- the library's chain)
//   k_step_correct  per cell labelled at n + 1 (unless the solid failed): xi^{n+1/2} =
//                   (xi^n + xi^{n+1}) / 2 where the cell was labelled at n too, else
//                   xi^{n+1}.
// Every kernel takes one 64-cell row segment per wave (the mask word of the segment).
// The arithmetic is evaluated per value in one fixed order without contraction (this
// file is compiled with -ffp-contract=off), so the predicted values, and with them the
// interior decisions, are those of any implementation of the same expressions.
// Memory-bound stencil work in FP64 on a thin set of cells: no MFMA.
#include "rmx_device.h"
#include "rmx_step.h"

namespace rmx {
namespace {
using namespace dev;

__device__ __forceinline__ double dmin2(double a, double b) { return a < b ? a : b; }

// Second-order limited slope at q0 from (qm, q0, qp).
__device__ __forceinline__ double slope2(double qm, double q0, double qp) {
    const double dl = q0 - qm, dr = qp - q0;
    if (!(dl * dr > 0.0)) return 0.0;
    const double dc = 0.5 * (qp - qm);
    const double m = dmin2(fabs(dc), 2.0 * dmin2(fabs(dl), fabs(dr)));
    return copysign(m, dc);
}

// Colella's fourth-order monotonicity-limited slope at q0 (difference per cell).
__device__ __forceinline__ double slope4(double qm2, double qm1, double q0, double qp1,
                                         double qp2) {
    const double dl = q0 - qm1, dr = qp1 - q0;
    if (!(dl * dr > 0.0)) return 0.0;
    const double dc = 0.5 * (qp1 - qm1);
    const double fp = slope2(q0, qp1, qp2), fm = slope2(qm2, qm1, q0);
    const double d4 = (4.0 / 3.0) * dc - (1.0 / 6.0) * (fp + fm);
    const double m = dmin2(fabs(d4), 2.0 * dmin2(fabs(dl), fabs(dr)));
    return copysign(m, dc);
}

// Loads of the step's arrays through the global address space (partial waits).
template <typename T>
__device__ __forceinline__ T ld(const T* p, int64_t i) {
    return load_global(p + i);
}

// Slope of field p at cell x along a stride s.
__device__ __forceinline__ double slope_at(const double* p, int64_t x, int64_t s) {
    return slope4(ld(p, x - 2 * s), ld(p, x - s), ld(p, x), ld(p, x + s), ld(p, x + 2 * s));
}

// Godunov choice of a transverse advecting velocity from its down and up expansions.
__device__ __forceinline__ double godunov_vel(double vd, double vu) {
    if (vd > 0.0 && vd + vu > 0.0) return vd;
    if (vu < 0.0 && vd + vu < 0.0) return vu;
    return 0.0;
}

// The left/down state if w > 0, the right/up state if w < 0, their mean if w = 0.
__device__ __forceinline__ double upwind(double w, double lo, double hi) {
    if (w > 0.0) return lo;
    if (w < 0.0) return hi;
    return 0.5 * (lo + hi);
}

__device__ __forceinline__ int find_solid_by_word(const DevSolid* s, int n, int64_t w) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s[mid].word_base <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t axis_stride(const DevSolid* d, int a) {
    return a == 0 ? 1 : (a == 1 ? (int64_t)d->n0 : (int64_t)d->n0 * d->n1);
}

// One wave's row segment: solid, local word, cell coordinates of this lane.
struct Seg {
    int s;
    int64_t lw;
    int i, j, k;
    int64_t c;
};

__device__ __forceinline__ Seg segment(const StepBatch& b, int64_t w) {
    Seg g;
    g.s = uniform_int(find_solid_by_word(b.solids, b.n_solids, w));
    const DevSolid* d = b.solids + g.s;
    g.lw = w - d->word_base;
    const int row = (int)(g.lw / d->W);
    const int wx = (int)(g.lw - (int64_t)row * d->W);
    g.k = row / d->n1;
    g.j = row - g.k * d->n1;
    g.i = wx * 64 + (int)(threadIdx.x & 63);
    g.c = ((int64_t)g.k * d->n1 + g.j) * d->n0 + g.i;
    return g;
}

__device__ __forceinline__ int64_t wave_segment() {
    return (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
}

// ------------------------------------------------------------------------------------
// Transverse faces.  Block 0 also zeroes the call's statistics and brick counters.
// ------------------------------------------------------------------------------------
__device__ void trans_segment(const StepBatch& b, int64_t w) {
    {
        const Seg g = segment(b, w);
        const DevSolid* d = b.solids + g.s;
        const StepDev* sd = b.steps + g.s;
        const int L = d->L;
        int lab = -1;
        if (g.i < d->n0) lab = ld(sd->labels_n, g.c);
        // faces that a predicted cell reads lie within L1 distance 2 of it
        const bool act = lab >= 0 && lab <= L - 2;
        if (__ballot(act) == 0ull) return;
        if (!act) return;
        const int64_t nc = d->ncell;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int ct = t == 0 ? g.i : (t == 1 ? g.j : g.k);
            const int nt = t == 0 ? d->n0 : (t == 1 ? d->n1 : d->n2);
            if (ct < 2 || ct > nt - 4) continue;
            const int64_t s = axis_stride(d, t);
            const int64_t x = g.c, y = g.c + s;
            const double hl = b.hl[t];
            const double* v = sd->u + t * nc;
            const double vx = ld(v, x), vy = ld(v, y);
            const double vd = vx + (0.5 - hl * vx) * slope_at(v, x, s);
            const double vu = vy - (0.5 + hl * vy) * slope_at(v, y, s);
            const double wv = godunov_vel(vd, vu);
            double* tr = sd->trans + (int64_t)t * 4 * nc;
            tr[x] = wv;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double* p = sd->xi_n + q * nc;
                const double qd = ld(p, x) + (0.5 - hl * vx) * slope_at(p, x, s);
                const double qu = ld(p, y) - (0.5 + hl * vy) * slope_at(p, y, s);
                tr[(1 + q) * nc + x] = upwind(wv, qd, qu);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_step_trans(StepBatch b) {
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < b.n_solids * kStatWords; i += 256) b.stats[i] = 0ull;
        for (int i = threadIdx.x; i < kMaxLayers * kBuckets; i += 256) b.bcount[i] = 0;
        const int nctl = (int)(sizeof(BandCtl) / sizeof(int));
        for (int i = threadIdx.x; i < nctl; i += 256) reinterpret_cast<int*>(b.band)[i] = 0;
    }
    const int64_t w = wave_segment();
    if (w < b.total_words) trans_segment(b, w);
}

// Tangential term along axis t at cell m, component q, without the 1/Delta_t: (mean of the
// transverse advecting velocities on the cell's two t-faces) x (difference of the chosen
// states).
__device__ __forceinline__ double tangential(const StepDev* sd, const DevSolid* d, int64_t m,
                                             int t, int q) {
    const int64_t nc = d->ncell;
    const int64_t s = axis_stride(d, t);
    const double* tr = sd->trans + (int64_t)t * 4 * nc;
    const double wm = ld(tr, m - s), wp = ld(tr, m);
    const double qm = ld(tr, (1 + q) * nc + m - s), qp = ld(tr, (1 + q) * nc + m);
    return (0.5 * (wm + wp)) * (qp - qm);
}

// Expansion of component q from cell x to its +a face (side = 0, the left state of that
// face) or to its -a face (side = 1, the right state of that face); hl = dt / (2 Delta_a),
// tang = the tangential terms of the other two axes, each times its dt / (2 Delta_t).
__device__ __forceinline__ double side_state(const StepDev* sd, const DevSolid* d, double hl,
                                             int64_t x, int a, int q, int side, double tang) {
    const int64_t nc = d->ncell;
    const int64_t s = axis_stride(d, a);
    const double* ua = sd->u + a * nc;
    const double* p = sd->xi_n + q * nc;
    const double sl = slope_at(p, x, s);
    if (side == 0) return (ld(p, x) + (0.5 - hl * ld(ua, x)) * sl) - tang;
    return (ld(p, x) - (0.5 + hl * ld(ua, x)) * sl) - tang;
}

// Face-normal velocity on the low face of cell (i, j, k) along axis a.
__device__ __forceinline__ double face_vel(const StepDev* sd, const DevSolid* d, int a, int i,
                                           int j, int k) {
    const int64_t n0 = d->n0, n1 = d->n1;
    if (a == 0) return ld(sd->uf[0], ((int64_t)k * n1 + j) * (n0 + 1) + i);
    if (a == 1) return ld(sd->uf[1], ((int64_t)k * (n1 + 1) + j) * n0 + i);
    return ld(sd->uf[2], ((int64_t)k * n1 + j) * n0 + i);
}

// A predicted cell: labelled 0..L-4 at step n and 3 cells inside the box.
__device__ __forceinline__ bool predicted(const StepDev* sd, const DevSolid* d, int i, int j,
                                          int k) {
    if (i < 3 || i > d->n0 - 4 || j < 3 || j > d->n1 - 4 || k < 3 || k > d->n2 - 4)
        return false;
    const int lab = ld(sd->labels_n, ((int64_t)k * d->n1 + j) * d->n0 + i);
    return lab >= 0 && lab <= d->L - 4;
}

// ------------------------------------------------------------------------------------
// Side states: per cell next to a predicted cell and per axis, the expansions of xi to the
// cell's +a face (left state of that face) and -a face (right state of that face).
// faces[(a * 2 + side) * 3 + q][cell].
// ------------------------------------------------------------------------------------
__device__ void faces_segment(const StepBatch& b, int64_t w) {
    const Seg g = segment(b, w);
    const DevSolid* d = b.solids + g.s;
    const StepDev* sd = b.steps + g.s;
    int lab = -1;
    if (g.i < d->n0) lab = ld(sd->labels_n, g.c);
    // a cell whose face a predicted cell reads is within L1 distance 1 of it
    const bool act = lab >= 0 && lab <= d->L - 3;
    if (__ballot(act) == 0ull) return;
    if (!act) return;
    const int64_t nc = d->ncell;
    const bool self = predicted(sd, d, g.i, g.j, g.k);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // +a face: read by this cell or by its +a neighbour; -a face: by this cell or by its
        // -a neighbour
        const bool hi = self || predicted(sd, d, g.i + (a == 0), g.j + (a == 1), g.k + (a == 2));
        const bool lo = self || predicted(sd, d, g.i - (a == 0), g.j - (a == 1), g.k - (a == 2));
        if (!hi && !lo) continue;
        const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        const double hl = b.hl[a], h1 = b.hl[t1], h2 = b.hl[t2];
#pragma unroll 1
        for (int q = 0; q < 3; ++q) {
            const double tang =
                h1 * tangential(sd, d, g.c, t1, q) + h2 * tangential(sd, d, g.c, t2, q);
            if (hi)
                sd->faces[(int64_t)((a * 2 + 0) * 3 + q) * nc + g.c] =
                    side_state(sd, d, hl, g.c, a, q, 0, tang);
            if (lo)
                sd->faces[(int64_t)((a * 2 + 1) * 3 + q) * nc + g.c] =
                    side_state(sd, d, hl, g.c, a, q, 1, tang);
        }
    }
}

__global__ __launch_bounds__(256) void k_step_faces(StepBatch b) {
    const int64_t w = wave_segment();
    if (w < b.total_words) faces_segment(b, w);
}

// ------------------------------------------------------------------------------------
// Predictor and the interior mask of step n + 1.
// ------------------------------------------------------------------------------------
__device__ void predict_segment(const StepBatch& b, int64_t w) {
    const double l0 = b.lam[0], l1 = b.lam[1], l2 = b.lam[2];
    const int lane = threadIdx.x & 63;
    const Seg g = segment(b, w);
    const DevSolid* d = b.solids + g.s;
    const StepDev* sd = b.steps + g.s;
    const int L = d->L;
    const int n0 = d->n0, n1 = d->n1, n2 = d->n2;
    const int64_t nc = d->ncell;
    int lab = -1;
    if (g.i < n0) lab = ld(sd->labels_n, g.c);
    const bool inb =
        g.i >= 3 && g.i <= n0 - 4 && g.j >= 3 && g.j <= n1 - 4 && g.k >= 3 && g.k <= n2 - 4;
    const bool pred = lab >= 0 && lab <= L - 4 && inb;
    const bool other = lab >= 0 && lab <= L && !pred;
    bool inside = false;
    if (__ballot(lab >= 0) != 0ull) {
        if (pred) {
            double um[3], up[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                um[a] = face_vel(sd, d, a, g.i, g.j, g.k);
                up[a] = face_vel(sd, d, a, g.i + (a == 0), g.j + (a == 1), g.k + (a == 2));
            }
            double nv[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                double term[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int64_t s = axis_stride(d, a);
                    const double* fl = sd->faces + (int64_t)((a * 2 + 0) * 3 + q) * nc;
                    const double* fr = sd->faces + (int64_t)((a * 2 + 1) * 3 + q) * nc;
                    // -a face: left state from cell c - e_a, right state from c
                    const double xm = upwind(um[a], ld(fl, g.c - s), ld(fr, g.c));
                    // +a face: left state from c, right state from c + e_a
                    const double xp = upwind(up[a], ld(fl, g.c), ld(fr, g.c + s));
                    term[a] = (0.5 * (um[a] + up[a])) * (xp - xm);
                }
                const double acc = (l0 * term[0] + l1 * term[1]) + l2 * term[2];
                nv[q] = ld(sd->xi_n, q * nc + g.c) - acc;
                d->xi[q * nc + g.c] = nv[q];
            }
            inside = interior(load_shape(d), nv[0], nv[1], nv[2]);
        } else if (other) {
#pragma unroll
            for (int q = 0; q < 3; ++q) d->xi[q * nc + g.c] = __builtin_nan("");
        }
    }
    const unsigned long long m = __ballot(inside);
    const unsigned long long lost = __ballot(other && lab == 0);
    if (lane == 0) {
        d->mask[g.lw] = m;
        if (lost) atomicOr(b.stats + (int64_t)g.s * kStatWords + ST_FLAGS, FLAG_TRUNCATED);
    }
}

__global__ __launch_bounds__(256) void k_step_predict(StepBatch b) {
    const int64_t w = wave_segment();
    if (w < b.total_words) predict_segment(b, w);
}

// ------------------------------------------------------------------------------------
// Corrector.
// ------------------------------------------------------------------------------------
__device__ void correct_segment(const StepBatch& b, int64_t w) {
    {
        const Seg g = segment(b, w);
        const DevSolid* d = b.solids + g.s;
        const StepDev* sd = b.steps + g.s;
        const unsigned long long fl = b.stats[(int64_t)g.s * kStatWords + ST_FLAGS];
        if (fl & (FLAG_TRUNCATED | FLAG_OVERFLOW | FLAG_TIMEOUT)) return;   // uniform
        const int L = d->L;
        if (g.i >= d->n0) return;
        const int ln = ld(d->labels, g.c);
        if (ln < 0 || ln > L) return;
        const int lo = ld(sd->labels_n, g.c);
        const bool both = lo >= 0 && lo <= L;
        const int64_t nc = d->ncell;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double a = ld(d->xi, q * nc + g.c);
            sd->xi_half[q * nc + g.c] = both ? (ld(sd->xi_n, q * nc + g.c) + a) * 0.5 : a;
        }
    }
}

__global__ __launch_bounds__(256) void k_step_correct(StepBatch b) {
    const int64_t w = wave_segment();
    if (w < b.total_words) correct_segment(b, w);
}

// One row segment per wave, four waves per block.  (Eight segments per wave, scanned with
// one round of label loads, measured slower: a wave then works through the active
// segments of the dense interior one after another.)
int step_grid(const StepBatch& b) {
    const int64_t blocks = (b.total_words + 3) / 4;
    return (int)(blocks > 0 ? blocks : 1);
}

}  // namespace

hipError_t launch_step_trans(const StepBatch& b, hipStream_t st) {
    hipLaunchKernelGGL(k_step_trans, dim3(step_grid(b)), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_step_faces(const StepBatch& b, hipStream_t st) {
    hipLaunchKernelGGL(k_step_faces, dim3(step_grid(b)), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_step_predict(const StepBatch& b, hipStream_t st) {
    hipLaunchKernelGGL(k_step_predict, dim3(step_grid(b)), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_step_correct(const StepBatch& b, hipStream_t st) {
    hipLaunchKernelGGL(k_step_correct, dim3(step_grid(b)), dim3(256), 0, st, b);
    return hipGetLastError();
}

}  // namespace rmx
