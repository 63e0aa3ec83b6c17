/*
 * rmx_oracle.c -- plain CPU oracle for the layer-wise weighted-least-squares (WLS)
 * extrapolation of the reference map xi, as defined in Lin, Derr & Rycroft,
 * "Eulerian simulation of complex suspensions and biolocomotion in three dimensions":
 *   - main text, section "Extrapolation of xi(x,t)" (layer labelling, layer order,
 *     eligible data, local linear model, degeneracy rule, object independence);
 *   - SI, section "Weighting scheme for weighted least squares-based extrapolation",
 *     equation (weight);
 *   - main text, "Blurred interface method": phi(x,t) = phi0(xi(x,t)), phi0 a signed
 *     distance in reference coordinates; interior cells are those with phi < 0;
 *   - SI "Variable arrangement" (spacings Delta x, Delta y, Delta z of the M x N x O
 *     cells) and SI "Test cases" (periodic domains).
 *
 * Readings of the last two: the fit's offsets stay in cells (an affine model's value at
 * the target does not change when its columns are scaled), and only the normal factor of
 * eq. (weight) sees the spacings, through the physical x' and gradient.  A solid's box
 * holds its unwrapped map; along a periodic axis the box may run past the grid's end
 * (the caller wraps it onto the grid), and no box face there is a wall.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path loads this file: only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg do.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * It is written to be checked by eye against the paper, not to be fast:
 *   classify every cell, label layers by a FIFO breadth-first search, then for each layer
 *   in ascending order fit each cell on its own with a Householder QR of the weighted
 *   design matrix.  OpenMP only splits the independent cells of one layer.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC  (no FMA contraction anywhere,
 * so the interior predicate, the signed distance and the weight sign test are evaluated
 * exactly in the written order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Status codes (same numeric values as the library's documented codes). */
#define ORC_OK 0
#define ORC_W_EMPTY 1
#define ORC_E_ARG (-1)
#define ORC_E_BOX (-2)
#define ORC_E_LAYERS (-3)
#define ORC_E_SHAPE (-4)
#define ORC_E_TRUNCATED (-7)

/* Decision codes written per cell. */
#define ORC_DEC_F1 32          /* normal factor dropped at r_max                 */
#define ORC_DEC_F2 33          /* plain kernel-weighted mean at r_max            */
#define ORC_DEC_NO_NORMAL 64   /* added when l <= normal_layers but grad phi = 0 */

#define ORC_MAX_LAYERS 16
#define ORC_MAX_R 8

typedef struct {
    int32_t kind;       /* 1 = sphere, 2 = ellipsoid                                   */
    double centre[3];   /* in reference coordinates                                    */
    double semi[3];     /* semi-axes; a sphere uses semi[0] as its radius              */
    double rot[9];      /* row-major 3x3; column a is body axis a in reference coords  */
} orc_shape;

typedef struct {
    int32_t grid_n[3];      /* M, N, O cells of the whole grid                        */
    int32_t lo[3], ext[3];  /* the solid's box inside the grid                         */
    orc_shape shape;
    int32_t n_layers;       /* L                                                      */
    int32_t r_s, r_max;     /* search radius and its cap                              */
    int32_t normal_layers;  /* eq. (weight) uses the normal for layers <= this (2)    */
    int32_t adjacency;      /* 6: face neighbours; 26: every cell of the 3^3 cube      */
    int32_t periodic[3];    /* 1: the grid is periodic along this axis (no walls)      */
    double spacing[3];      /* Delta x, Delta y, Delta z ("Variable arrangement")      */
} orc_problem;

/* stats layout (int64): [0] interior, [1..16] band cells of layer l, [17] cells whose
 * radius grew, [18] cells with no normal, [19] F1 cells, [20] F2 cells.             */
#define ORC_N_STATS 21

/* ------------------------------------------------------------------------------------
 * phi0 and the interior predicate ("Blurred interface method"; "Extrapolation of xi").
 * ---------------------------------------------------------------------------------- */

/* Body coordinates y = rot^T (v - centre), summed in the fixed order (b = 0, 1, 2). */
static void body_coords(const orc_shape* s, const double v[3], double y[3]) {
    double d0 = v[0] - s->centre[0];
    double d1 = v[1] - s->centre[1];
    double d2 = v[2] - s->centre[2];
    for (int a = 0; a < 3; ++a)
        y[a] = (s->rot[0 * 3 + a] * d0 + s->rot[1 * 3 + a] * d1) + s->rot[2 * 3 + a] * d2;
}

static int all_finite(const double v[3]) {
    return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

/* A cell is interior when phi0(xi) < 0 (strictly).  The sign is decided without a
 * square root: |xi - c|^2 < R^2 for a sphere, the quadratic form q < 1 for an
 * ellipsoid.  A cell whose xi has a non-finite component is undefined, never interior. */
static int is_interior(const orc_shape* s, const double v[3]) {
    if (!all_finite(v)) return 0;
    if (s->kind == 1) {
        double dx = v[0] - s->centre[0];
        double dy = v[1] - s->centre[1];
        double dz = v[2] - s->centre[2];
        double r = s->semi[0];
        return ((dx * dx + dy * dy) + dz * dz) < r * r;
    }
    double y[3];
    body_coords(s, v, y);
    double q0 = y[0] / s->semi[0], q1 = y[1] / s->semi[1], q2 = y[2] / s->semi[2];
    return ((q0 * q0 + q1 * q1) + q2 * q2) < 1.0;
}

/* F(s) = sum over coordinates with u_a > 0 of (e_a u_a / (s + d_a))^2 - 1, where
 * s = t + e_m^2 is the Lagrange multiplier measured from the pole of the shortest axis m
 * among those coordinates and d_a = e_a^2 - e_m^2 >= 0. */
static double ell_F(const double e[3], const double dd[3], const double u[3], double s) {
    double f = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (u[a] > 0.0) {
            double q = (e[a] * u[a]) / (s + dd[a]);
            f = f + q * q;
        }
    }
    return f - 1.0;
}

/* Euclidean distance from the point y (body coordinates) to the ellipsoid surface
 * sum (x_a/e_a)^2 = 1.  The closest point x satisfies x_a (t + e_a^2) = e_a^2 y_a for a
 * Lagrange multiplier t >= -min_a e_a^2.  On the coordinates with y_a != 0, t is the
 * unique root of sum (e_a y_a / (t + e_a^2))^2 = 1 above -e_m^2 (m: shortest such axis).
 * The root is sought in s = t + e_m^2, bracketed by [e_m |y_m|, |(e_a y_a)_a|], by
 * bisection until the midpoint equals an end of the bracket; working in s keeps full
 * relative precision when the root lies extremely close to the pole (tiny |y_m|).  When
 * every coordinate along the shortest axes is exactly zero, the closest point may leave
 * that coordinate plane (t = -e_min^2), which is tested first. */
static double ell_distance(const double e[3], const double y[3]) {
    double u[3] = {fabs(y[0]), fabs(y[1]), fabs(y[2])};
    double e2[3] = {e[0] * e[0], e[1] * e[1], e[2] * e[2]};
    int amin = 0;
    for (int a = 1; a < 3; ++a)
        if (e[a] < e[amin]) amin = a;
    int m = -1;
    for (int a = 0; a < 3; ++a)
        if (u[a] > 0.0 && (m < 0 || e[a] < e[m])) m = a;
    if (m < 0) return e[amin]; /* the centre: nearest points lie on the shortest axis */

    if (e[m] > e[amin]) {
        double S = 0.0, D = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (u[a] > 0.0) {
                double x = (e2[a] * u[a]) / (e2[a] - e2[amin]);
                double q = x / e[a];
                S = S + q * q;
                D = D + (x - u[a]) * (x - u[a]);
            }
        }
        if (S < 1.0) return sqrt(D + e2[amin] * (1.0 - S));
    }

    double dd[3], sq = 0.0;
    for (int a = 0; a < 3; ++a) {
        dd[a] = e2[a] - e2[m];
        if (u[a] > 0.0) {
            double p = e[a] * u[a];
            sq = sq + p * p;
        }
    }
    double s0 = e[m] * u[m];
    double s1 = sqrt(sq);
    for (int it = 0; it < 4096; ++it) {
        double sm = 0.5 * (s0 + s1);
        if (sm <= s0 || sm >= s1) break;
        double f = ell_F(e, dd, u, sm);
        if (f > 0.0)
            s0 = sm;
        else if (f < 0.0)
            s1 = sm;
        else {
            s0 = sm;
            s1 = sm;
            break;
        }
    }
    double s = 0.5 * (s0 + s1);
    double D = 0.0;
    for (int a = 0; a < 3; ++a) {
        double x = (u[a] > 0.0) ? (e2[a] * u[a]) / (s + dd[a]) : 0.0;
        D = D + (x - u[a]) * (x - u[a]);
    }
    return sqrt(D);
}

/* phi0(v): signed distance to the reference surface, negative inside.  The sign comes
 * from the interior predicate so that it agrees with the labelling exactly. */
static double phi0_eval(const orc_shape* s, const double v[3]) {
    double dist;
    if (s->kind == 1) {
        double dx = v[0] - s->centre[0];
        double dy = v[1] - s->centre[1];
        double dz = v[2] - s->centre[2];
        dist = fabs(sqrt((dx * dx + dy * dy) + dz * dz) - s->semi[0]);
    } else {
        double y[3];
        body_coords(s, v, y);
        dist = ell_distance(s->semi, y);
    }
    return is_interior(s, v) ? -dist : dist;
}

/* ------------------------------------------------------------------------------------
 * Box indexing.  xi is SoA [3][ext2][ext1][ext0]; labels are [ext2][ext1][ext0].
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int64_t n0, n1, n2, ncell;
} box_dims;

static box_dims dims_of(const orc_problem* p) {
    box_dims b;
    b.n0 = p->ext[0];
    b.n1 = p->ext[1];
    b.n2 = p->ext[2];
    b.ncell = b.n0 * b.n1 * b.n2;
    return b;
}

static int64_t cell_index(const box_dims* b, int64_t i, int64_t j, int64_t k) {
    return (k * b->n1 + j) * b->n0 + i;
}

static void load_xi(const double* xi, const box_dims* b, int64_t c, double v[3]) {
    v[0] = xi[c];
    v[1] = xi[b->ncell + c];
    v[2] = xi[2 * b->ncell + c];
}

static int check_problem(const orc_problem* p) {
    for (int a = 0; a < 3; ++a) {
        if (p->grid_n[a] <= 0 || p->ext[a] <= 0) return ORC_E_ARG;
        if (!(p->spacing[a] > 0.0) || !isfinite(p->spacing[a])) return ORC_E_ARG;
        if (p->periodic[a]) {
            /* the box starts inside the grid and may run past its end (it wraps), but it
             * never covers a cell twice */
            if (p->lo[a] < 0 || p->lo[a] >= p->grid_n[a] || p->ext[a] > p->grid_n[a])
                return ORC_E_BOX;
        } else if (p->lo[a] < 0 || p->lo[a] + p->ext[a] > p->grid_n[a]) {
            return ORC_E_BOX;
        }
    }
    if (p->n_layers < 0 || p->n_layers > ORC_MAX_LAYERS) return ORC_E_LAYERS;
    if (p->r_s < 1 || p->r_max < p->r_s || p->r_max > ORC_MAX_R) return ORC_E_ARG;
    if (p->normal_layers < 0) return ORC_E_ARG;
    if (p->adjacency != 6 && p->adjacency != 26) return ORC_E_ARG;
    if (p->shape.kind != 1 && p->shape.kind != 2) return ORC_E_SHAPE;
    int na = (p->shape.kind == 1) ? 1 : 3;
    for (int a = 0; a < na; ++a)
        if (!(p->shape.semi[a] > 0.0) || !isfinite(p->shape.semi[a])) return ORC_E_SHAPE;
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------
 * Layer labelling ("Extrapolation of xi", first paragraph; Fig. 1(c)):
 * interior cells are layer 0; every unmarked face neighbour of a layer-(l-1) cell becomes
 * layer l, up to L; growth stops at the grid walls.  Implemented literally as a FIFO
 * breadth-first search.  With adjacency 26 (the same section's remark that layers follow
 * from any adjacency on the grid) the neighbours are the 26 cells of the 3^3 cube.  Returns the number of interior cells, or a negative status.
 * ---------------------------------------------------------------------------------- */
int64_t orc_label(const orc_problem* p, const double* xi, int8_t* labels, int32_t* truncated) {
    int st = check_problem(p);
    if (st != ORC_OK) return st;
    box_dims b = dims_of(p);
    int L = p->n_layers;
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)b.ncell);
    if (!queue) return ORC_E_ARG;
    int64_t head = 0, tail = 0, n_int = 0;
    int trunc = 0;
    for (int64_t c = 0; c < b.ncell; ++c) {
        double v[3];
        load_xi(xi, &b, c, v);
        if (is_interior(&p->shape, v)) {
            labels[c] = 0;
            queue[tail++] = c;
            ++n_int;
            /* The band of an interior cell closer than L to a box face that is not a grid
             * wall would leave the box.  A periodic axis has no walls: there the box must
             * hold the whole band (its fields are the unwrapped map of the solid). */
            int64_t ii = c % b.n0, jj = (c / b.n0) % b.n1, kk = c / (b.n0 * b.n1);
            int64_t idx[3] = {ii, jj, kk};
            for (int a = 0; a < 3; ++a) {
                int low_wall = !p->periodic[a] && p->lo[a] == 0;
                int high_wall = !p->periodic[a] && p->lo[a] + p->ext[a] == p->grid_n[a];
                if (!low_wall && idx[a] < L) trunc = 1;
                if (!high_wall && (p->ext[a] - 1 - idx[a]) < L) trunc = 1;
            }
        } else {
            labels[c] = -1;
        }
    }
    while (head < tail) {
        int64_t c = queue[head++];
        int lc = labels[c];
        if (lc >= L) continue;
        int64_t i = c % b.n0, j = (c / b.n0) % b.n1, k = c / (b.n0 * b.n1);
        /* the neighbours under the problem's adjacency: offsets with |d|_1 = 1 (faces),
         * or every non-zero offset of the 3^3 cube */
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    int n1 = (di != 0) + (dj != 0) + (dk != 0);
                    if (n1 == 0 || (p->adjacency == 6 && n1 != 1)) continue;
                    int64_t x = i + di, y = j + dj, z = k + dk;
                    if (x < 0 || x >= b.n0 || y < 0 || y >= b.n1 || z < 0 || z >= b.n2)
                        continue;
                    int64_t d = cell_index(&b, x, y, z);
                    if (labels[d] == -1) {
                        labels[d] = (int8_t)(lc + 1);
                        queue[tail++] = d;
                    }
                }
    }
    free(queue);
    if (truncated) *truncated = trunc;
    return n_int;
}

/* ------------------------------------------------------------------------------------
 * Normal at a band cell (SI, weighting scheme): gradient of phi0(xi) by differences of
 * the face neighbours in the given field; central where both neighbours are defined and
 * inside the box, else one-sided with the cell itself (forward first), else 0.
 * In differences per cell: the physical gradient divides component a by Delta_a, which
 * the weight does.
 * ---------------------------------------------------------------------------------- */
static int phi_at(const orc_problem* p, const box_dims* b, const double* field, int64_t i,
                  int64_t j, int64_t k, double* out) {
    if (i < 0 || i >= b->n0 || j < 0 || j >= b->n1 || k < 0 || k >= b->n2) return 0;
    double v[3];
    load_xi(field, b, cell_index(b, i, j, k), v);
    if (!all_finite(v)) return 0;
    *out = phi0_eval(&p->shape, v);
    return 1;
}

static void normal_at(const orc_problem* p, const box_dims* b, const double* field,
                      int64_t i, int64_t j, int64_t k, double g[3]) {
    double pe = 0.0;
    int de = phi_at(p, b, field, i, j, k, &pe);
    for (int a = 0; a < 3; ++a) {
        int64_t sp[3] = {i, j, k}, sm[3] = {i, j, k};
        sp[a] += 1;
        sm[a] -= 1;
        double vp = 0.0, vm = 0.0;
        int dp = phi_at(p, b, field, sp[0], sp[1], sp[2], &vp);
        int dm = phi_at(p, b, field, sm[0], sm[1], sm[2], &vm);
        if (dp && dm)
            g[a] = 0.5 * (vp - vm);
        else if (dp && de)
            g[a] = vp - pe;
        else if (dm && de)
            g[a] = pe - vm;
        else
            g[a] = 0.0;
    }
}

/* ------------------------------------------------------------------------------------
 * Exact degeneracy test: the WLS system [1, delta] over the data with positive weight has
 * full rank 4 iff those integer offsets are not all coplanar.  Greedy search for a second
 * distinct point, a third off their line and a fourth off their plane, in integers.
 * ---------------------------------------------------------------------------------- */
static int full_affine_rank(int n, const int32_t (*pts)[3]) {
    if (n < 4) return 0;
    int64_t v1[3] = {0, 0, 0}, cr[3] = {0, 0, 0};
    int stage = 0;
    for (int q = 1; q < n; ++q) {
        int64_t d[3] = {pts[q][0] - pts[0][0], pts[q][1] - pts[0][1], pts[q][2] - pts[0][2]};
        if (stage == 0) {
            if (d[0] || d[1] || d[2]) {
                v1[0] = d[0];
                v1[1] = d[1];
                v1[2] = d[2];
                stage = 1;
            }
        } else if (stage == 1) {
            int64_t c0 = v1[1] * d[2] - v1[2] * d[1];
            int64_t c1 = v1[2] * d[0] - v1[0] * d[2];
            int64_t c2 = v1[0] * d[1] - v1[1] * d[0];
            if (c0 || c1 || c2) {
                cr[0] = c0;
                cr[1] = c1;
                cr[2] = c2;
                stage = 2;
            }
        } else {
            if (cr[0] * d[0] + cr[1] * d[1] + cr[2] * d[2] != 0) return 1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Weighted least squares by Householder QR.  Rows: sqrt(w) [1, dx, dy, dz] and
 * sqrt(w) xi_d.  Returns beta_0 (the affine model evaluated at the target, i.e. at
 * delta = 0) for the three components.
 * ---------------------------------------------------------------------------------- */
static void wls_qr(int n, double (*A)[4], double (*B)[3], double out[3]) {
    for (int col = 0; col < 4; ++col) {
        double tail2 = 0.0;
        for (int r = col + 1; r < n; ++r) tail2 += A[r][col] * A[r][col];
        double norm = sqrt(A[col][col] * A[col][col] + tail2);
        double alpha = (A[col][col] > 0.0) ? -norm : norm;
        double v0 = A[col][col] - alpha;
        /* Householder vector v = (v0, A[col+1..n-1][col]); H = I - 2 v v^T / (v^T v). */
        double vtv = v0 * v0 + tail2;
        if (vtv == 0.0) continue;
        for (int c2 = col + 1; c2 < 4; ++c2) {
            double s = v0 * A[col][c2];
            for (int r = col + 1; r < n; ++r) s += A[r][col] * A[r][c2];
            double f = 2.0 * s / vtv;
            A[col][c2] -= f * v0;
            for (int r = col + 1; r < n; ++r) A[r][c2] -= f * A[r][col];
        }
        for (int c2 = 0; c2 < 3; ++c2) {
            double s = v0 * B[col][c2];
            for (int r = col + 1; r < n; ++r) s += A[r][col] * B[r][c2];
            double f = 2.0 * s / vtv;
            B[col][c2] -= f * v0;
            for (int r = col + 1; r < n; ++r) B[r][c2] -= f * A[r][col];
        }
        A[col][col] = alpha;
        for (int r = col + 1; r < n; ++r) A[r][col] = 0.0;
    }
    /* Back substitution R beta = (Q^T B)[0:4]. */
    double beta[4][3];
    for (int c2 = 0; c2 < 3; ++c2) {
        for (int row = 3; row >= 0; --row) {
            double s = B[row][c2];
            for (int q = row + 1; q < 4; ++q) s -= A[row][q] * beta[q][c2];
            beta[row][c2] = s / A[row][row];
        }
        out[c2] = beta[0][c2];
    }
}

/* One band cell e = (i, j, k) of layer le.  Writes its new xi (into `res`) and returns
 * its decision code.  `labels` holds the final labels; `xi` holds interior values and
 * the values of layers < le already extrapolated. */
static int fit_cell(const orc_problem* p, const box_dims* b, const double* xi,
                    const int8_t* labels, int64_t i, int64_t j, int64_t k, int le,
                    int has_normal, const double g[3], double res[3]) {
    const int rmax = p->r_max;
    const int nmax = (2 * rmax + 1) * (2 * rmax + 1) * (2 * rmax + 1);
    double(*A)[4] = malloc(sizeof(double[4]) * (size_t)nmax);
    double(*B)[3] = malloc(sizeof(double[3]) * (size_t)nmax);
    int32_t(*P)[3] = malloc(sizeof(int32_t[3]) * (size_t)nmax);
    double* W = malloc(sizeof(double) * (size_t)nmax);
    int64_t* D = malloc(sizeof(int64_t) * (size_t)nmax);
    /* the physical gradient of phi0(xi) and its length */
    double gp[3];
    for (int a = 0; a < 3; ++a) gp[a] = g[a] / p->spacing[a];
    double gn = sqrt((gp[0] * gp[0] + gp[1] * gp[1]) + gp[2] * gp[2]);
    int code = -1;

    /* Pass 0..: radii r_s..r_max with eq. (weight); then F1 (kernel only) at r_max. */
    for (int pass = 0; pass <= (rmax - p->r_s) + 1 && code < 0; ++pass) {
        int f1 = (pass == rmax - p->r_s + 1);
        if (f1 && !has_normal) break; /* F1 would repeat the last pass exactly */
        int r = f1 ? rmax : p->r_s + pass;
        int use_normal = has_normal && !f1;
        int n = 0;
        for (int dz = -r; dz <= r; ++dz)
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    int64_t ii = i + dx, jj = j + dy, kk = k + dz;
                    if (ii < 0 || ii >= b->n0 || jj < 0 || jj >= b->n1 || kk < 0 || kk >= b->n2)
                        continue;
                    int64_t d = cell_index(b, ii, jj, kk);
                    int ld = labels[d];
                    if (!(ld >= 0 && ld < le)) continue; /* eligible data only */
                    double base = ldexp(1.0, -(abs(dx) + abs(dy) + abs(dz)));
                    double w;
                    if (use_normal) {
                        /* x' = x_e - x_d = -(dx Delta_x, dy Delta_y, dz Delta_z), physical.
                         * x'.n > 0 iff delta . g < 0 (the spacings cancel between x' and
                         * the physical gradient), decided on this exact expression; the
                         * cosine's magnitude comes from the physical vectors. */
                        double fx = (double)dx, fy = (double)dy, fz = (double)dz;
                        double dot = (fx * g[0] + fy * g[1]) + fz * g[2];
                        if (!(dot < 0.0)) continue;
                        double px = fx * p->spacing[0], py = fy * p->spacing[1],
                               pz = fz * p->spacing[2];
                        double pdot = (px * gp[0] + py * gp[1]) + pz * gp[2];
                        double dlen = sqrt((px * px + py * py) + pz * pz);
                        w = (fabs(pdot) / (dlen * gn)) * base;
                    } else {
                        w = base;
                    }
                    P[n][0] = dx;
                    P[n][1] = dy;
                    P[n][2] = dz;
                    W[n] = w;
                    D[n] = d;
                    ++n;
                }
        if (full_affine_rank(n, (const int32_t(*)[3])P)) {
            for (int q = 0; q < n; ++q) {
                double sw = sqrt(W[q]);
                A[q][0] = sw;
                A[q][1] = sw * P[q][0];
                A[q][2] = sw * P[q][1];
                A[q][3] = sw * P[q][2];
                double v[3];
                load_xi(xi, b, D[q], v);
                B[q][0] = sw * v[0];
                B[q][1] = sw * v[1];
                B[q][2] = sw * v[2];
            }
            wls_qr(n, A, B, res);
            code = f1 ? ORC_DEC_F1 : r;
        }
    }
    if (code < 0) {
        /* F2: kernel-weighted mean over the eligible data at r_max.  Never empty: the
         * face neighbour the cell was labelled from is eligible. */
        double sw = 0.0, s[3] = {0.0, 0.0, 0.0};
        for (int dz = -rmax; dz <= rmax; ++dz)
            for (int dy = -rmax; dy <= rmax; ++dy)
                for (int dx = -rmax; dx <= rmax; ++dx) {
                    int64_t ii = i + dx, jj = j + dy, kk = k + dz;
                    if (ii < 0 || ii >= b->n0 || jj < 0 || jj >= b->n1 || kk < 0 || kk >= b->n2)
                        continue;
                    int64_t d = cell_index(b, ii, jj, kk);
                    int ld = labels[d];
                    if (!(ld >= 0 && ld < le)) continue;
                    double base = ldexp(1.0, -(abs(dx) + abs(dy) + abs(dz)));
                    double v[3];
                    load_xi(xi, b, d, v);
                    sw += base;
                    s[0] += base * v[0];
                    s[1] += base * v[1];
                    s[2] += base * v[2];
                }
        res[0] = s[0] / sw;
        res[1] = s[1] / sw;
        res[2] = s[2] / sw;
        code = ORC_DEC_F2;
    }
    free(A);
    free(B);
    free(P);
    free(W);
    free(D);
    return code;
}

/* ------------------------------------------------------------------------------------
 * Whole extrapolation of one solid: classify, label, then layers 1..L in ascending order
 * ("Extrapolation of xi", second paragraph), cells of one layer independent.  xi is
 * updated in place on band cells only; interior and unmarked cells are left untouched.
 * xi_normal (nullable) is the field the normals are taken from; NULL means the input xi
 * as it was at the start of the call.  decisions (nullable) receives one code per cell.
 * ---------------------------------------------------------------------------------- */
int orc_extrapolate(const orc_problem* p, double* xi, const double* xi_normal,
                    int8_t* labels, int8_t* decisions, int64_t* stats, int32_t nthreads) {
    int st = check_problem(p);
    if (st != ORC_OK) return st;
    box_dims b = dims_of(p);
    int L = p->n_layers;
    int64_t st_local[ORC_N_STATS];
    memset(st_local, 0, sizeof(st_local));
    if (decisions) memset(decisions, 0, (size_t)b.ncell);

    int32_t trunc = 0;
    int64_t n_int = orc_label(p, xi, labels, &trunc);
    if (n_int < 0) return (int)n_int;
    st_local[0] = n_int;
    for (int64_t c = 0; c < b.ncell; ++c)
        if (labels[c] > 0) st_local[labels[c]] += 1;
    int status = ORC_OK;
    if (trunc)
        status = ORC_E_TRUNCATED;
    else if (n_int == 0)
        status = ORC_W_EMPTY;
    if (status != ORC_OK || L == 0) {
        if (stats) memcpy(stats, st_local, sizeof(st_local));
        return status;
    }

    const double* nfield = xi_normal;
    double* copy = NULL;
    if (!nfield && p->normal_layers > 0) {
        copy = (double*)malloc(sizeof(double) * 3 * (size_t)b.ncell);
        memcpy(copy, xi, sizeof(double) * 3 * (size_t)b.ncell);
        nfield = copy;
    }

    int64_t* cells = (int64_t*)malloc(sizeof(int64_t) * (size_t)b.ncell);
    double* res = (double*)malloc(sizeof(double) * 3 * (size_t)b.ncell);
    int8_t* codes = (int8_t*)malloc((size_t)b.ncell);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int l = 1; l <= L; ++l) {
        int64_t nl = 0;
        for (int64_t c = 0; c < b.ncell; ++c)
            if (labels[c] == l) cells[nl++] = c;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t q = 0; q < nl; ++q) {
            int64_t c = cells[q];
            int64_t i = c % b.n0, j = (c / b.n0) % b.n1, k = c / (b.n0 * b.n1);
            double g[3] = {0.0, 0.0, 0.0};
            int has_normal = 0, no_normal = 0;
            if (l <= p->normal_layers) {
                normal_at(p, &b, nfield, i, j, k, g);
                has_normal = (g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0);
                no_normal = !has_normal;
            }
            int code = fit_cell(p, &b, xi, labels, i, j, k, l, has_normal, g, &res[3 * q]);
            codes[q] = (int8_t)(code + (no_normal ? ORC_DEC_NO_NORMAL : 0));
        }
        /* Cells of one layer read only layers < l, so the writes can follow the layer. */
        for (int64_t q = 0; q < nl; ++q) {
            int64_t c = cells[q];
            xi[c] = res[3 * q];
            xi[b.ncell + c] = res[3 * q + 1];
            xi[2 * b.ncell + c] = res[3 * q + 2];
            int code = codes[q];
            if (decisions) decisions[c] = (int8_t)code;
            int base_code = code & ~ORC_DEC_NO_NORMAL;
            if (code & ORC_DEC_NO_NORMAL) st_local[18] += 1;
            if (base_code == ORC_DEC_F1) st_local[19] += 1;
            if (base_code == ORC_DEC_F2) st_local[20] += 1;
            if (base_code == ORC_DEC_F1 || base_code == ORC_DEC_F2 || base_code > p->r_s)
                st_local[17] += 1;
        }
    }
    free(cells);
    free(res);
    free(codes);
    free(copy);
    if (stats) memcpy(stats, st_local, sizeof(st_local));
    return ORC_OK;
}

/* Exported single evaluations, for the tests that pin the pieces. */
double orc_phi0(const orc_shape* s, double x, double y, double z) {
    double v[3] = {x, y, z};
    return phi0_eval(s, v);
}

int orc_is_interior(const orc_shape* s, double x, double y, double z) {
    double v[3] = {x, y, z};
    return is_interior(s, v);
}

int orc_full_rank(int32_t n, const int32_t* pts) {
    return full_affine_rank(n, (const int32_t(*)[3])pts);
}

/* Normal g (unnormalised) at box cell (i, j, k) from `field`. */
void orc_normal(const orc_problem* p, const double* field, int32_t i, int32_t j, int32_t k,
                double* g) {
    box_dims b = dims_of(p);
    normal_at(p, &b, field, i, j, k, g);
}
