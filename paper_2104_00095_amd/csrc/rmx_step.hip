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
// A scan lists the 64-cell row segments (mask words) with a labelled cell, at step n
// before the predictor and at n + 1 before the corrector; every other kernel then takes
// one listed segment per wave, so a launch spans the thin band, not the box.
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

// Field p at cells x and x + s, and its slopes there: the six values x - 2s .. x + 3s are
// loaded once.
struct Pair {
    double vx, vy, sx, sy;
};

__device__ __forceinline__ Pair pair_at(const double* p, int64_t x, int64_t s) {
    const double m2 = ld(p, x - 2 * s), m1 = ld(p, x - s), c0 = ld(p, x), p1 = ld(p, x + s),
                 p2 = ld(p, x + 2 * s), p3 = ld(p, x + 3 * s);
    return {c0, p1, slope4(m2, m1, c0, p1, p2), slope4(m1, c0, p1, p2, p3)};
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

// upwind() on stored states, loading only the state(s) the sign of w selects.
__device__ __forceinline__ double upwind_ld(double w, const double* plo, int64_t ilo,
                                            const double* phi, int64_t ihi) {
    if (w > 0.0) return load_global(plo + ilo);
    if (w < 0.0) return load_global(phi + ihi);
    return 0.5 * (load_global(plo + ilo) + load_global(phi + ihi));
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
// The scan: 16 row segments per wave, their labels loaded together; a segment with a cell
// labelled 0..L joins the list.  A block appends its segments with one atomic to its
// sub-list, in segment order.  At step n (which = 0) block 0 also zeroes the call's
// statistics and brick counters, and every segment's interior mask word is zeroed (the
// predictor writes the listed ones).
// ------------------------------------------------------------------------------------
constexpr int kScanWords = kStepScanWords / 4;

__device__ void scan_append(const StepBatch& b, int which, unsigned act, int lane, int wid,
                            int64_t w0);

__global__ __launch_bounds__(256) void k_step_scan(StepBatch b, int which) {
    if (which == 0 && blockIdx.x == 0) {
        for (int i = threadIdx.x; i < b.n_solids * kStatWords; i += 256) b.stats[i] = 0ull;
        for (int i = threadIdx.x; i < kMaxLayers * kBuckets; i += 256) b.bcount[i] = 0;
        const int nctl = (int)(sizeof(BandCtl) / sizeof(int));
        for (int i = threadIdx.x; i < nctl; i += 256) reinterpret_cast<int*>(b.band)[i] = 0;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t w0 = wave_segment() * kScanWords;
    unsigned act = 0u;   // bit u: segment w0 + u is listed (the same in every lane)
    // Whole rows of whole segments (n0 a multiple of 64, 16-byte aligned labels): the
    // wave's 16 segments are 1 KB of consecutive labels, 16 bytes per lane, tested four at
    // a time for a byte below L + 1 (unsigned: -1 is 255).
    if (w0 < b.total_words) {
        const int s = uniform_int(find_solid_by_word(b.solids, b.n_solids, w0));
        const DevSolid* d = b.solids + s;
        const int8_t* lp = which == 0 ? b.steps[s].labels_n : d->labels;
        const int64_t lw0 = w0 - d->word_base;
        const int64_t nw = (int64_t)d->W * d->n1 * d->n2;
        if (d->n0 == 64 * d->W && lw0 + kScanWords <= nw &&
            (reinterpret_cast<uintptr_t>(lp) & 15) == 0) {
            const uint4 v = reinterpret_cast<const uint4*>(lp + lw0 * 64)[lane];
            const unsigned n = 0x01010101u * (unsigned)(d->L + 1);
            const auto below = [n](unsigned x) { return ((x - n) & ~x & 0x80808080u) != 0u; };
            const bool f = below(v.x) || below(v.y) || below(v.z) || below(v.w);
            const unsigned long long m = __ballot(f);
#pragma unroll
            for (int u = 0; u < kScanWords; ++u)
                if ((m >> (4 * u)) & 0xFull) act |= 1u << u;
            if (which == 0 && lane < kScanWords) d->mask[lw0 + lane] = 0ull;
            scan_append(b, which, act, lane, wid, w0);
            return;
        }
    }
    int lab[kScanWords];
    // the wave's segments are consecutive: the first one's place is computed, the rest
    // follow by steps (a new solid is located again)
    // (the solid's fields are held in registers: the mask stores could alias them)
    const int8_t* lp = nullptr;
    unsigned long long* mask = nullptr;
    int64_t end_w = 0, lw = 0;
    int wx = 0, j = 0, k = 0, n0 = 0, n1 = 0, W = 1, L = 0;
#pragma unroll
    for (int u = 0; u < kScanWords; ++u) {
        lab[u] = -1;
        const int64_t w = w0 + u;
        if (w >= b.total_words) continue;   // uniform
        if (w >= end_w) {
            const int s = uniform_int(find_solid_by_word(b.solids, b.n_solids, w));
            const DevSolid* d = b.solids + s;
            lp = which == 0 ? b.steps[s].labels_n : d->labels;
            mask = d->mask;
            n0 = d->n0;
            n1 = d->n1;
            W = d->W;
            L = d->L;
            end_w = d->word_base + (int64_t)W * n1 * d->n2;
            lw = w - d->word_base;
            const int row = (int)(lw / W);
            wx = (int)(lw - (int64_t)row * W);
            k = row / n1;
            j = row - k * n1;
        }
        const int i = wx * 64 + lane;
        if (i < n0) {
            const int l = ld(lp, ((int64_t)k * n1 + j) * n0 + i);
            lab[u] = l <= L ? l : -1;
        }
        if (which == 0 && lane == 0) mask[lw] = 0ull;
        ++lw;
        if (++wx == W) {
            wx = 0;
            if (++j == n1) {
                j = 0;
                ++k;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kScanWords; ++u) {
        if (w0 + u >= b.total_words) break;   // uniform
        if (__ballot(lab[u] >= 0)) act |= 1u << u;
    }
    scan_append(b, which, act, lane, wid, w0);
}

// A block's listed segments (bits of each wave's act) appended to its sub-list with one
// atomic, in segment order.
__device__ void scan_append(const StepBatch& b, int which, unsigned act, int lane, int wid,
                            int64_t w0) {
    __shared__ int s_cnt[4];
    __shared__ int s_base;
    if (lane == 0) s_cnt[wid] = __builtin_popcount(act);
    __syncthreads();
    const int x = blockIdx.x % kStepLists;
    if (threadIdx.x == 0) {
        const int tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        s_base = tot ? atomicAdd(&b.counts[which * kStepLists + x], tot) : 0;
    }
    __syncthreads();
    if (lane == 0 && act) {
        int pos = s_base;
        for (int v = 0; v < wid; ++v) pos += s_cnt[v];
        int32_t* list = b.lists + (int64_t)(which * kStepLists + x) * b.list_cap;
        for (int u = 0; u < kScanWords; ++u)
            if ((act >> u) & 1u) list[pos++] = (int32_t)(w0 + u);
    }
}

// A listed kernel: wave i of the launch takes entries i, i + waves, ... of the
// concatenated sub-lists.
#define STEP_LIST_LOOP(which, body)                                                     \
    do {                                                                                \
        int pre_[kStepLists + 1];                                                       \
        pre_[0] = 0;                                                                    \
        for (int x_ = 0; x_ < kStepLists; ++x_)                                         \
            pre_[x_ + 1] = pre_[x_] + b.counts[(which) * kStepLists + x_];               \
        for (int i_ = (int)wave_segment(); i_ < pre_[kStepLists]; i_ += gridDim.x * 4) { \
            int x_ = 0;                                                                 \
            while (i_ >= pre_[x_ + 1]) ++x_;                                            \
            const int32_t* list_ = b.lists + (int64_t)((which) * kStepLists + x_) * b.list_cap; \
            body(b, (int64_t)list_[i_ - pre_[x_]]);                                     \
        }                                                                               \
    } while (0)

// ------------------------------------------------------------------------------------
// Transverse faces.
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
            const int64_t x = g.c;
            const double hl = b.hl[t];
            const Pair v = pair_at(sd->u + t * nc, x, s);
            const double vx = v.vx, vy = v.vy;
            const double vd = vx + (0.5 - hl * vx) * v.sx;
            const double vu = vy - (0.5 + hl * vy) * v.sy;
            const double wv = godunov_vel(vd, vu);
            double* tr = sd->trans + (int64_t)t * 4 * nc;
            tr[x] = wv;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                // only the expansion the sign of wv selects (both where it is 0)
                const double* p = sd->xi_n + q * nc;
                double v;
                if (wv > 0.0) {
                    v = ld(p, x) + (0.5 - hl * vx) * slope_at(p, x, s);
                } else if (wv < 0.0) {
                    v = ld(p, x + s) - (0.5 + hl * vy) * slope_at(p, x + s, s);
                } else {
                    const Pair pq = pair_at(p, x, s);
                    const double qd = pq.vx + (0.5 - hl * vx) * pq.sx;
                    const double qu = pq.vy - (0.5 + hl * vy) * pq.sy;
                    v = upwind(wv, qd, qu);
                }
                tr[(1 + q) * nc + x] = v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_step_trans(StepBatch b) {
    STEP_LIST_LOOP(0, trans_segment);
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
        // ... and only the side the face velocity's sign selects there (both where it is 0)
        const bool hi =
            (self || predicted(sd, d, g.i + (a == 0), g.j + (a == 1), g.k + (a == 2))) &&
            !(face_vel(sd, d, a, g.i + (a == 0), g.j + (a == 1), g.k + (a == 2)) < 0.0);
        const bool lo =
            (self || predicted(sd, d, g.i - (a == 0), g.j - (a == 1), g.k - (a == 2))) &&
            !(face_vel(sd, d, a, g.i, g.j, g.k) > 0.0);
        if (!hi && !lo) continue;
        const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        const double hl = b.hl[a], h1 = b.hl[t1], h2 = b.hl[t2];
        const int64_t s = axis_stride(d, a);
        const double ux = ld(sd->u + a * nc, g.c);
        // Tangential terms along t1 and t2, each without its 1/Delta_t: (mean of the
        // transverse advecting velocities on the cell's two t-faces, shared by the three
        // components) x (difference of the chosen states)
        const int64_t s1 = axis_stride(d, t1), s2 = axis_stride(d, t2);
        const double* tr1 = sd->trans + (int64_t)t1 * 4 * nc;
        const double* tr2 = sd->trans + (int64_t)t2 * 4 * nc;
        const double w1 = 0.5 * (ld(tr1, g.c - s1) + ld(tr1, g.c));
        const double w2 = 0.5 * (ld(tr2, g.c - s2) + ld(tr2, g.c));
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double* q1 = tr1 + (1 + q) * nc;
            const double* q2 = tr2 + (1 + q) * nc;
            const double tang = h1 * (w1 * (ld(q1, g.c) - ld(q1, g.c - s1))) +
                                h2 * (w2 * (ld(q2, g.c) - ld(q2, g.c - s2)));
            // both sides share the cell's value, slope and tangential terms
            const double* p = sd->xi_n + q * nc;
            const double sl = slope_at(p, g.c, s), px = ld(p, g.c);
            if (hi)
                sd->faces[(int64_t)((a * 2 + 0) * 3 + q) * nc + g.c] =
                    (px + (0.5 - hl * ux) * sl) - tang;
            if (lo)
                sd->faces[(int64_t)((a * 2 + 1) * 3 + q) * nc + g.c] =
                    (px - (0.5 + hl * ux) * sl) - tang;
        }
    }
}

__global__ __launch_bounds__(256) void k_step_faces(StepBatch b) {
    STEP_LIST_LOOP(0, faces_segment);
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
                    const double xm = upwind_ld(um[a], fl, g.c - s, fr, g.c);
                    // +a face: left state from c, right state from c + e_a
                    const double xp = upwind_ld(up[a], fl, g.c, fr, g.c + s);
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
    STEP_LIST_LOOP(0, predict_segment);
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
    STEP_LIST_LOOP(1, correct_segment);
}

// Listed kernels: four waves per block, one listed segment per wave at a time, at most
// kStepBlocks blocks (a list never exceeds the box's segments).  (Eight segments per
// wave, one after another, measured slower: a wave then works through the active segments
// of the dense interior in turn.)
constexpr int64_t kStepBlocks = 4096;

int step_grid(const StepBatch& b) {
    int64_t blocks = (b.total_words + 3) / 4;
    if (blocks > kStepBlocks) blocks = kStepBlocks;
    return (int)(blocks > 0 ? blocks : 1);
}

}  // namespace

hipError_t launch_step_scan(const StepBatch& b, int which, hipStream_t st) {
    const int64_t blocks = (b.total_words + kStepScanWords - 1) / kStepScanWords;
    hipLaunchKernelGGL(k_step_scan, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                       st, b, which);
    return hipGetLastError();
}

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
