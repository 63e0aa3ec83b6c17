/*
 * rmx_blur_oracle.c -- plain CPU oracle for the blur-zone consumers of the extrapolated
 * reference maps, as defined in Lin, Derr & Rycroft, "Eulerian simulation of complex
 * suspensions and biolocomotion in three dimensions" (arXiv 2104.00095):
 *   - main text, "Blurred interface method and monolithic governing equations":
 *     phi(x) = phi0(xi(x)); the smoothed Heaviside of eq. (sm_heavi);
 *   - SI, "Stress calculations": the deformation gradient F = (grad_x xi)^{-1} at the cell
 *     faces by centred differences of the reference map, B = F F^T, the incompressible
 *     neo-Hookean stress tau_s = G (B - tr(B)/3 I) per solid, the blend of the solid
 *     stresses of overlapping blur zones with the weights 1 - H_eps(phi_m), and the
 *     multi-body modified Heaviside of eq. (mod_heaviside).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path loads this file: only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg do.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Readings (where the paper is silent), listed in the design notes as well:
 *   - a solid covers a cell of its box labelled 0..L (interior or band): there phi_m is
 *     phi0_m(xi_m); elsewhere it contributes nothing (its blur zone must lie inside its
 *     band: L is chosen from eps);
 *   - the modified Heaviside is written on every grid cell inside some solid's box;
 *     cells outside every box are left as the caller had them (pure fluid, H = 1);
 *   - at a face between cells P (low) and Q (high) along axis a, d xi / d x_a is
 *     (xi(Q) - xi(P)) / Delta_a, and d xi / d x_t (t != a) is the mean of the centred
 *     differences at P and Q: ((xi(P+t) - xi(P-t)) + (xi(Q+t) - xi(Q-t))) / (4 Delta_t),
 *     with the spacings Delta of SI "Variable arrangement"; the solid contributes at the
 *     face only where all these cells lie in its box and are labelled 0..L;
 *   - phi_m at a face is phi0_m of the face value of xi, (xi(P) + xi(Q)) / 2;
 *   - the blended stress is written on every face with a cell inside some solid's box
 *     (zero where no solid contributes); other faces are left as they were;
 *   - periodic domains (SI "Test cases"): a box holds the solid's unwrapped map and may
 *     run past the end of a periodic axis; its local cell l covers grid cell
 *     (lo + l) mod n there.  The difference stencil is taken in the box, so it never
 *     joins the two ends of a box that spans the whole axis.  A periodic axis has n
 *     faces (face i between cells i - 1 mod n and i), a walled one n + 1.
 * Sums over solids run in increasing solid index.  Stress components are stored in the
 * order xx, yy, zz, xy, xz, yz.
 *
 * Build: with the other oracle files, gcc -O2 -ffp-contract=off (no contraction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int32_t kind;
    double centre[3];
    double semi[3];
    double rot[9];
} orb_shape;   /* the oracle's shape layout (same fields as in rmx_oracle.c) */

double orc_phi0(const orb_shape* s, double x, double y, double z);

typedef struct {
    int32_t lo[3], ext[3];
    orb_shape shape;
    int32_t n_layers;
    const double* xi;       /* [3][e2][e1][e0] */
    const int8_t* labels;   /* [e2][e1][e0]    */
} orb_solid;

/* Smoothed Heaviside, eq. (sm_heavi). */
double orc_heaviside_eps(double phi, double eps) {
    if (phi <= -eps) return 0.0;
    if (phi >= eps) return 1.0;
    return 0.5 * ((1.0 + phi / eps) + sin(M_PI * phi / eps) / M_PI);
}

typedef struct {
    int64_t n[3];
    int32_t periodic[3];
} orb_grid;

/* Box coordinates of global cell g in solid s's box: 1 if it lies there, else 0. */
static int box_coords(const orb_grid* G, const orb_solid* s, const int64_t g[3], int64_t l[3]) {
    for (int a = 0; a < 3; ++a) {
        int64_t d = g[a] - s->lo[a];
        if (G->periodic[a]) d = ((d % G->n[a]) + G->n[a]) % G->n[a];
        if (d < 0 || d >= s->ext[a]) return 0;
        l[a] = d;
    }
    return 1;
}

/* Index of the cell at box coordinates l, or -1 outside the box. */
static int64_t box_cell(const orb_solid* s, const int64_t l[3]) {
    for (int a = 0; a < 3; ++a)
        if (l[a] < 0 || l[a] >= s->ext[a]) return -1;
    return (l[2] * s->ext[1] + l[1]) * s->ext[0] + l[0];
}

/* Index in solid s's box of global cell g, or -1 outside it. */
static int64_t local_cell(const orb_grid* G, const orb_solid* s, const int64_t g[3]) {
    int64_t l[3];
    if (!box_coords(G, s, g, l)) return -1;
    return box_cell(s, l);
}

static int covered(const orb_solid* s, int64_t c) {
    int lab = s->labels[c];
    return lab >= 0 && lab <= s->n_layers;
}

static void xi_at(const orb_solid* s, int64_t c, double v[3]) {
    int64_t nc = (int64_t)s->ext[0] * s->ext[1] * s->ext[2];
    for (int q = 0; q < 3; ++q) v[q] = s->xi[q * nc + c];
}

/* Modified Heaviside, eq. (mod_heaviside): H = max(1 - sum_m (1 - H_eps(phi_m)), 0) on
 * every grid cell inside some box.  phi (nullable; entries nullable) receives phi_m on the
 * cells of solid m's box labelled 0..L. */
void orc_blur(const int32_t grid_n[3], const int32_t periodic[3], int32_t n_solids,
              const orb_solid* solids, double eps, double* H, double* const* phi) {
    orb_grid G = {{grid_n[0], grid_n[1], grid_n[2]}, {periodic[0], periodic[1], periodic[2]}};
    for (int64_t k = 0; k < grid_n[2]; ++k)
        for (int64_t j = 0; j < grid_n[1]; ++j)
            for (int64_t i = 0; i < grid_n[0]; ++i) {
                int64_t g[3] = {i, j, k};
                int any = 0;
                double acc = 0.0;
                for (int m = 0; m < n_solids; ++m) {
                    const orb_solid* s = &solids[m];
                    int64_t c = local_cell(&G, s, g);
                    if (c < 0) continue;
                    any = 1;
                    if (!covered(s, c)) continue;
                    double v[3];
                    xi_at(s, c, v);
                    double p = orc_phi0(&s->shape, v[0], v[1], v[2]);
                    if (phi && phi[m]) phi[m][c] = p;
                    acc += 1.0 - orc_heaviside_eps(p, eps);
                }
                if (!any) continue;
                double d = 1.0 - acc;
                H[(k * grid_n[1] + j) * grid_n[0] + i] = d > 0.0 ? d : 0.0;
            }
}

/* Neo-Hookean stress of solid s at the face between the cells at box coordinates
 * P = q - e_a and Q = q; returns 0 (no contribution) unless the whole difference stencil
 * is covered.  h: the spacings. */
static int face_stress(const orb_solid* s, const int64_t q[3], int a, const double h[3],
                       double G, double tau[6], double* w, double eps) {
    int64_t P[3] = {q[0], q[1], q[2]}, Q[3] = {q[0], q[1], q[2]};
    P[a] -= 1;
    int64_t cp = box_cell(s, P), cq = box_cell(s, Q);
    if (cp < 0 || cq < 0 || !covered(s, cp) || !covered(s, cq)) return 0;
    double xp[3], xq[3];
    xi_at(s, cp, xp);
    xi_at(s, cq, xq);
    double J[3][3];   /* J[q][b] = d xi_q / d x_b */
    for (int c = 0; c < 3; ++c) J[c][a] = (xq[c] - xp[c]) / h[a];
    for (int t = 0; t < 3; ++t) {
        if (t == a) continue;
        int64_t Pm[3] = {P[0], P[1], P[2]}, Pp[3] = {P[0], P[1], P[2]};
        int64_t Qm[3] = {Q[0], Q[1], Q[2]}, Qp[3] = {Q[0], Q[1], Q[2]};
        Pm[t] -= 1; Pp[t] += 1; Qm[t] -= 1; Qp[t] += 1;
        int64_t c1 = box_cell(s, Pm), c2 = box_cell(s, Pp);
        int64_t c3 = box_cell(s, Qm), c4 = box_cell(s, Qp);
        if (c1 < 0 || c2 < 0 || c3 < 0 || c4 < 0) return 0;
        if (!covered(s, c1) || !covered(s, c2) || !covered(s, c3) || !covered(s, c4)) return 0;
        double v1[3], v2[3], v3[3], v4[3];
        xi_at(s, c1, v1); xi_at(s, c2, v2); xi_at(s, c3, v3); xi_at(s, c4, v4);
        for (int c = 0; c < 3; ++c) J[c][t] = ((v2[c] - v1[c]) + (v4[c] - v3[c])) / (4.0 * h[t]);
    }
    /* F = J^{-1} by cofactors */
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = (J[0][0] * c00 + J[0][1] * c01) + J[0][2] * c02;
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
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[r][c] = (F[r][0] * F[c][0] + F[r][1] * F[c][1]) + F[r][2] * F[c][2];
    double tr3 = ((B[0][0] + B[1][1]) + B[2][2]) / 3.0;
    tau[0] = G * (B[0][0] - tr3);
    tau[1] = G * (B[1][1] - tr3);
    tau[2] = G * (B[2][2] - tr3);
    tau[3] = G * B[0][1];
    tau[4] = G * B[0][2];
    tau[5] = G * B[1][2];
    double xf[3];
    for (int c = 0; c < 3; ++c) xf[c] = (xp[c] + xq[c]) * 0.5;
    *w = 1.0 - orc_heaviside_eps(orc_phi0(&s->shape, xf[0], xf[1], xf[2]), eps);
    return 1;
}

/* Blended solid stress at the faces (SI "Stress calculations"): with S = sum_m w_m and
 * T = sum_m w_m tau_m, the face gets T if S <= 1, T / S otherwise.  tau[a] is
 * [6][n2 + f2][n1 + f1][n0 + f0] with f_b = 1 if b == a and axis a is walled, else 0.
 * h: the spacings Delta_x, Delta_y, Delta_z.  G: one shear modulus per solid. */
void orc_solid_stress(const int32_t grid_n[3], const int32_t periodic[3], int32_t n_solids,
                      const orb_solid* solids, double eps, const double h[3], const double* G,
                      double* const tau[3]) {
    orb_grid Gr = {{grid_n[0], grid_n[1], grid_n[2]}, {periodic[0], periodic[1], periodic[2]}};
    for (int a = 0; a < 3; ++a) {
        int64_t n[3] = {grid_n[0], grid_n[1], grid_n[2]};
        if (!periodic[a]) n[a] += 1;   /* faces along a */
        int64_t nf = n[0] * n[1] * n[2];
        for (int64_t k = 0; k < n[2]; ++k)
            for (int64_t j = 0; j < n[1]; ++j)
                for (int64_t i = 0; i < n[0]; ++i) {
                    int64_t g[3] = {i, j, k};
                    int64_t P[3] = {i, j, k};
                    P[a] -= 1;   /* the face's low cell (wrapped on a periodic axis) */
                    if (periodic[a] && P[a] < 0) P[a] += grid_n[a];
                    int any = 0;
                    double S = 0.0, T[6] = {0, 0, 0, 0, 0, 0};
                    for (int m = 0; m < n_solids; ++m) {
                        const orb_solid* s = &solids[m];
                        int64_t lq[3], lp[3];
                        int inq = g[a] < grid_n[a] && box_coords(&Gr, s, g, lq);
                        int inp = P[a] >= 0 && box_coords(&Gr, s, P, lp);
                        if (!inq && !inp) continue;
                        any = 1;
                        /* the face seen from the box: Q's box coordinates, or P's plus
                         * one step along a */
                        int64_t q[3];
                        for (int b = 0; b < 3; ++b) q[b] = inq ? lq[b] : lp[b];
                        if (!inq) q[a] += 1;
                        double t6[6], w;
                        if (!face_stress(s, q, a, h, G[m], t6, &w, eps)) continue;
                        S += w;
                        for (int c = 0; c < 6; ++c) T[c] += w * t6[c];
                    }
                    if (!any) continue;
                    int64_t f = (k * n[1] + j) * n[0] + i;
                    for (int c = 0; c < 6; ++c) tau[a][c * nf + f] = S <= 1.0 ? T[c] : T[c] / S;
                }
    }
}
