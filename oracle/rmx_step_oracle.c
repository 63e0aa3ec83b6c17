/*
 * rmx_step_oracle.c -- plain CPU oracle for the time-step coupling around the
 * extrapolation, as defined in Lin, Derr & Rycroft, "Eulerian simulation of complex
 * suspensions and biolocomotion in three dimensions" (arXiv 2104.00095):
 *   - SI, "Timestepping algorithm": step 5 (predictor of the primary reference maps
 *     xi^{n+1} from eq. (dis_xi_adv)), step 6 (extrapolation, done by rmx_oracle.c),
 *     step 7 (corrector xi^{n+1/2} = (xi^n + xi^{n+1}) / 2 on every available reference
 *     map) and step 11 (restore xi^{n+1}: the caller keeps xi^{n+1} in its own buffer);
 *   - SI, "Evaluating the advective term": eq. (adv_terms) for [(u.grad) xi]^{n+1/2};
 *     the Taylor-expanded face states of xi (eq. (xi_taylor_final) and its left-side
 *     companion); "Godunov-type upwinding scheme" (choice of a face state by the sign of
 *     the face velocity, the mean of both when it is zero); "Normal derivatives"
 *     (Colella's fourth-order monotonicity-limited slopes); "Tangential derivatives"
 *     (transverse face states without tangential terms, a Godunov choice of the
 *     transverse advecting velocity, and the centred difference of the chosen states).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path loads this file: only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg do.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Readings (where the paper is silent or defers to other work), listed in the design
 * notes as well:
 *   - the limited slope is Colella's fourth-order form: with dL = q0 - q-1, dR = q1 - q0,
 *     dc = (q1 - q-1) / 2 and the second-order limited slopes f(m) at the neighbours,
 *     slope = sign(dc) min(|4/3 dc - (f(1) + f(-1)) / 6|, 2|dL|, 2|dR|) where dL dR > 0,
 *     else 0; f(m) = sign(dc_m) min(|dc_m|, 2|dL_m|, 2|dR_m|) where dL_m dR_m > 0, else 0;
 *   - the face state of xi is chosen by the sign of the given face-normal velocity (the
 *     caller's advecting velocity at n + 1/2), which also advects in eq. (adv_terms);
 *   - the transverse expansions use the cell-centred velocity u^n and its own limited
 *     slope along the transverse axis;
 *   - the predictor runs on cells labelled 0..L-4 at step n that are at least 3 cells
 *     from every box face: there every value its face states read is a defined reference
 *     map of the labelled band (the stencil reaches 3 cells along an axis and L1 distance
 *     4).  The rest of the old band becomes undefined (NaN); unmarked cells are left as
 *     they are.  An interior cell closer than 3 cells to a box face cannot be predicted:
 *     the solid is reported truncated;
 *   - the corrector averages where the cell is labelled (0..L) at both steps, and takes
 *     xi^{n+1} where it is labelled only at step n + 1.
 *
 * Everything is evaluated per cell, on the fly, in the order written here (no FMA
 * contraction: built with -ffp-contract=off).  Lengths are in cells: with the spacing
 * Delta_a of axis a ("Variable arrangement"), lambda_a = dt / Delta_a and hl_a =
 * lambda_a / 2, (Delta_a/2 - dt u_a/2) d xi / d x_a = (1/2 - hl_a u_a) S for a per-cell
 * slope S along a, and dt/2 times the tangential term along t is hl_t times (mean
 * transverse velocity) x (difference of the transverse states).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n0, n1, n2, ncell;
} sbox;

static int64_t sidx(const sbox* b, int64_t i, int64_t j, int64_t k) {
    return (k * b->n1 + j) * b->n0 + i;
}

/* Offset of one cell step along axis a. */
static int64_t sstep(const sbox* b, int a) {
    return a == 0 ? 1 : (a == 1 ? b->n0 : b->n0 * b->n1);
}

static double dmin(double a, double b) { return a < b ? a : b; }

/* Second-order limited slope at the centre of q[-1..1] (q points at the centre). */
static double slope2(const double* q, int64_t s) {
    double dl = q[0] - q[-s], dr = q[s] - q[0];
    if (!(dl * dr > 0.0)) return 0.0;
    double dc = 0.5 * (q[s] - q[-s]);
    double m = dmin(fabs(dc), 2.0 * dmin(fabs(dl), fabs(dr)));
    return copysign(m, dc);
}

/* Colella's fourth-order monotonicity-limited slope at the centre of q[-2..2]
 * ("Normal derivatives"), a difference per cell. */
static double slope4(const double* q, int64_t s) {
    double dl = q[0] - q[-s], dr = q[s] - q[0];
    if (!(dl * dr > 0.0)) return 0.0;
    double dc = 0.5 * (q[s] - q[-s]);
    double fp = slope2(q + s, s), fm = slope2(q - s, s);
    double d4 = (4.0 / 3.0) * dc - (1.0 / 6.0) * (fp + fm);
    double m = dmin(fabs(d4), 2.0 * dmin(fabs(dl), fabs(dr)));
    return copysign(m, dc);
}

/* Godunov choice of a transverse advecting velocity from the down and up expansions. */
static double godunov_vel(double vd, double vu) {
    if (vd > 0.0 && vd + vu > 0.0) return vd;
    if (vu < 0.0 && vd + vu < 0.0) return vu;
    return 0.0;
}

/* A face value chosen by the sign of the advecting velocity w: left/down if w > 0,
 * right/up if w < 0, their mean if w = 0. */
static double upwind(double w, double lo, double hi) {
    if (w > 0.0) return lo;
    if (w < 0.0) return hi;
    return 0.5 * (lo + hi);
}

typedef struct {
    const sbox* b;
    const double* xi;   /* xi^n, SoA [3][ncell]             */
    const double* u;    /* cell velocity u^n, SoA [3][ncell] */
    double hl[3];       /* dt / (2 Delta_a) per axis          */
} sctx;

/* Transverse face of cell x along axis t, between x (down) and x + e_t (up)
 * ("Tangential derivatives"): the chosen advecting velocity and the chosen xi state
 * (component c). */
static void trans_face(const sctx* S, int64_t x, int t, int c, double* vadv, double* xib) {
    int64_t s = sstep(S->b, t);
    int64_t nc = S->b->ncell;
    const double* v = S->u + t * nc;   /* the t-component of the velocity */
    const double* q = S->xi + c * nc;
    double hl = S->hl[t];
    double vd = v[x] + (0.5 - hl * v[x]) * slope4(v + x, s);
    double vu = v[x + s] - (0.5 + hl * v[x + s]) * slope4(v + x + s, s);
    double w = godunov_vel(vd, vu);
    double qd = q[x] + (0.5 - hl * v[x]) * slope4(q + x, s);
    double qu = q[x + s] - (0.5 + hl * v[x + s]) * slope4(q + x + s, s);
    *vadv = w;
    *xib = upwind(w, qd, qu);
}

/* Tangential term along axis t at cell m for component c, without the 1/Delta_t:
 * (mean of the two transverse advecting velocities) x (difference of the two states). */
static double tangential(const sctx* S, int64_t m, int t, int c) {
    int64_t s = sstep(S->b, t);
    double wm, qm, wp, qp;
    trans_face(S, m - s, t, c, &wm, &qm);
    trans_face(S, m, t, c, &wp, &qp);
    return (0.5 * (wm + wp)) * (qp - qm);
}

/* Face state of component c on the face between x and x + e_a, chosen by the face
 * velocity uface (eq. (xi_taylor_final), its left-side companion, and the Godunov rule). */
static double normal_face(const sctx* S, int64_t x, int a, int c, double uface) {
    int64_t s = sstep(S->b, a);
    int64_t nc = S->b->ncell;
    const double* ua = S->u + a * nc;
    const double* q = S->xi + c * nc;
    int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;   /* the other two axes, ascending */
    const double* hl = S->hl;
    double left = (q[x] + (0.5 - hl[a] * ua[x]) * slope4(q + x, s)) -
                  (hl[t1] * tangential(S, x, t1, c) + hl[t2] * tangential(S, x, t2, c));
    int64_t y = x + s;
    double right = (q[y] - (0.5 + hl[a] * ua[y]) * slope4(q + y, s)) -
                   (hl[t1] * tangential(S, y, t1, c) + hl[t2] * tangential(S, y, t2, c));
    return upwind(uface, left, right);
}

/* Face-normal velocity on the low face of cell (i, j, k) along axis a: uf[a] holds
 * [n2][n1][n0+1] (a = 0), [n2][n1+1][n0] (a = 1), [n2+1][n1][n0] (a = 2). */
static double face_vel(const sbox* b, const double* const uf[3], int a, int64_t i, int64_t j,
                       int64_t k) {
    if (a == 0) return uf[0][(k * b->n1 + j) * (b->n0 + 1) + i];
    if (a == 1) return uf[1][(k * (b->n1 + 1) + j) * b->n0 + i];
    return uf[2][(k * b->n1 + j) * b->n0 + i];
}

/* Predictor (step 5, eq. (dis_xi_adv) with eq. (adv_terms)):
 * xi^{n+1} = xi^n - sum_a lambda_a [ (U_{a-} + U_{a+}) / 2 ] (Xi_{a+} - Xi_{a-}).
 * On the predicted cells (see the header) xi_next receives the value; on the rest of
 * the old band NaN; unmarked cells are left untouched.  Returns 1 if an interior cell
 * lies too close to a box face to be predicted, else 0. */
int orc_predict(const int32_t ext[3], int32_t n_layers, const double* xi_n,
                const int8_t* labels_n, const double* u, const double* ufx, const double* ufy,
                const double* ufz, const double lam[3], double* xi_next) {
    sbox b = {ext[0], ext[1], ext[2], (int64_t)ext[0] * ext[1] * ext[2]};
    const double* uf[3] = {ufx, ufy, ufz};
    sctx S = {&b, xi_n, u, {0.5 * lam[0], 0.5 * lam[1], 0.5 * lam[2]}};
    int trunc = 0;
    const int L = n_layers;
    for (int64_t k = 0; k < b.n2; ++k)
        for (int64_t j = 0; j < b.n1; ++j)
            for (int64_t i = 0; i < b.n0; ++i) {
                int64_t c = sidx(&b, i, j, k);
                int lab = labels_n[c];
                if (lab < 0 || lab > L) continue;
                int inside = i >= 3 && i <= b.n0 - 4 && j >= 3 && j <= b.n1 - 4 && k >= 3 &&
                             k <= b.n2 - 4;
                if (!(lab <= L - 4 && inside)) {
                    if (lab == 0) trunc = 1;
                    for (int q = 0; q < 3; ++q) xi_next[q * b.ncell + c] = NAN;
                    continue;
                }
                int64_t ijk[3] = {i, j, k};
                for (int q = 0; q < 3; ++q) {
                    double term[3];
                    for (int a = 0; a < 3; ++a) {
                        int64_t s = sstep(&b, a);
                        int64_t hi[3] = {ijk[0], ijk[1], ijk[2]};
                        hi[a] += 1;
                        double um = face_vel(&b, uf, a, i, j, k);
                        double up = face_vel(&b, uf, a, hi[0], hi[1], hi[2]);
                        double xm = normal_face(&S, c - s, a, q, um);
                        double xp = normal_face(&S, c, a, q, up);
                        term[a] = (0.5 * (um + up)) * (xp - xm);
                    }
                    double acc = (lam[0] * term[0] + lam[1] * term[1]) + lam[2] * term[2];
                    xi_next[q * b.ncell + c] = xi_n[q * b.ncell + c] - acc;
                }
            }
    return trunc;
}

/* Corrector (step 7): xi^{n+1/2} = (xi^n + xi^{n+1}) / 2 on cells labelled at both steps;
 * xi^{n+1} on cells labelled only at step n + 1; untouched elsewhere. */
void orc_correct(const int32_t ext[3], int32_t n_layers, const double* xi_n,
                 const int8_t* labels_n, const double* xi_next, const int8_t* labels_next,
                 double* xi_half) {
    int64_t nc = (int64_t)ext[0] * ext[1] * ext[2];
    for (int64_t c = 0; c < nc; ++c) {
        int ln = labels_next[c], lo = labels_n[c];
        if (ln < 0 || ln > n_layers) continue;
        int both = lo >= 0 && lo <= n_layers;
        for (int q = 0; q < 3; ++q) {
            double a = xi_next[q * nc + c];
            xi_half[q * nc + c] = both ? (xi_n[q * nc + c] + a) * 0.5 : a;
        }
    }
}

/* The limited slope alone, for the tests that pin it: q holds 5 values, centre q[2]. */
double orc_slope4(const double* q) { return slope4(q + 2, 1); }
