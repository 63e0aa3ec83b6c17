/*
 * rmx.h -- C ABI of the MI355X reference-map extrapolation library (librmx.so).
 *
 * The library extends the reference map xi of each solid from its interior cells into a
 * narrow band of fluid cells, one layer at a time, by the weighted-least-squares (WLS)
 * local linear fit of Lin, Derr & Rycroft, "Eulerian simulation of complex suspensions
 * and biolocomotion in three dimensions" (arXiv 2104.00095):
 *   - layers: main text, section "Extrapolation of xi(x,t)", first paragraph, and
 *     Fig. 1(c): interior cells (phi < 0) are layer 0; each unmarked face neighbour of a
 *     layer-(l-1) cell is layer l, until the grid wall or the layer count L;
 *   - fit: same section, second paragraph: layers in ascending order, cells of a layer
 *     independent; data are cells of the same object in lower layers within a box of
 *     radius r_s = 2; an affine model xi(x) ~ beta [1, x] evaluated at the target; a
 *     degenerate system grows r_s by one;
 *   - weights: SI section "Weighting scheme for weighted least squares-based
 *     extrapolation", eq. (weight): 2^-(|di|+|dj|+|dk|), times the non-negative cosine
 *     between x_e - x_d and the normalised gradient of phi0(xi) for layers <= 2;
 *   - phi(x) = phi0(xi(x)) with phi0 a signed distance in reference coordinates: main
 *     text, section "Blurred interface method and monolithic governing equations";
 *   - objects are extrapolated independently: same section of "Extrapolation of xi",
 *     third paragraph.
 * Readings where the paper is silent are fixed below and listed in the repository's
 * design notes: interior is phi0 < 0 strictly (a square-root-free predicate); the fit is
 * affine with an intercept, centred on the target; the search box is the Chebyshev cube
 * |d|_inf <= r; "degenerate" means the positive-weight offsets are coplanar (exact
 * integer test); r grows to r_max, then the normal factor is dropped (F1), then the
 * kernel-weighted mean is used (F2); the normal is taken from the field as it is at the
 * start of the call (or from xi_normal), by central differences of phi0(xi) over face
 * neighbours, one-sided where a neighbour is undefined or outside the box.
 *
 * Memory: every array argument marked DEVICE is a device pointer on the context's GPU,
 * owned by the caller, and must stay valid until the enqueued work has completed.  The
 * library owns its workspace.  All functions return an int status (RMX_OK = 0, > 0
 * warning, < 0 error).  Functions are thread-safe per context only if the caller
 * serialises calls on one context.
 */
#ifndef RMX_H
#define RMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
#define RMX_OK 0
#define RMX_W_EMPTY 1          /* solid has no interior cell: labels all -1, xi untouched */
#define RMX_E_ARG (-1)         /* null pointer, bad count or option out of range           */
#define RMX_E_BOX (-2)         /* box outside the grid or empty                            */
#define RMX_E_LAYERS (-3)      /* n_layers outside 0..RMX_MAX_LAYERS                       */
#define RMX_E_SHAPE (-4)       /* non-positive/non-finite semi-axis, non-orthonormal rot  */
#define RMX_E_WORKSPACE (-5)   /* fixed workspace too small for the call                   */
#define RMX_E_HIP (-6)         /* a HIP runtime call failed                                */
#define RMX_E_TRUNCATED (-7)   /* an interior cell lies within L of a box face that is not
                                  a grid wall: the band would leave the box.  Labels are
                                  written, xi is left untouched.                           */
#define RMX_E_BUDGET (-8)      /* server: request can never fit the HBM budget             */
#define RMX_E_BUSY (-9)        /* server: submission queue full                            */
#define RMX_E_NOTFOUND (-10)   /* server: unknown simulation or ticket                     */
#define RMX_E_DISABLED (-11)   /* the requested launch form is switched off in this build
                                  (no form is switched off at present)                     */

#define RMX_MAX_LAYERS 16
#define RMX_MAX_RADIUS 4

enum { RMX_SPHERE = 1, RMX_ELLIPSOID = 2 };
enum { RMX_FP64 = 0, RMX_FP32_ACCUM = 1 };

/* option flags */
#define RMX_FLAG_SYNC 1u       /* wait for completion and return the worst device status  */
#define RMX_FLAG_GRAPH 2u      /* capture the launch chain in a hipGraph and replay it on
                                  later calls with identical arguments                     */
#define RMX_FLAG_PER_SOLID 4u  /* plain form: one launch chain per solid, in order        */
#define RMX_FLAG_PROFILE 8u    /* record HIP events around every kernel of the chain (not
                                  with RMX_FLAG_GRAPH); read with rmx_profile_read         */
#define RMX_FLAG_PERSISTENT 16u /* the band work of the whole batch -- the normals and the
                                  fits of every layer, over the compacted brick lists -- in
                                  ONE persistent launch (after the classification and the
                                  labelling, two dense launches): blocks take bricks by
                                  ticket from per-XCD queues in layer order, and an item of
                                  layer l waits (bounded) until layer l - 1 is complete.  A
                                  wait that runs out reports RMX_E_HIP for the call.       */

#define RMX_FLAG_ADJ26 32u     /* layers by the 26-neighbour adjacency ("Extrapolation of
                                  xi", advantage (1): layers follow from any adjacency on the
                                  grid): every unmarked cell sharing a face, an edge or a
                                  corner with a layer-(l-1) cell is layer l, so the label is
                                  the Chebyshev distance to the interior (face neighbours,
                                  the default, give the L1 distance).  The fit is unchanged. */

/* Kernel phases reported by rmx_profile_read. */
#define RMX_PHASE_CLASSIFY 0
#define RMX_PHASE_LABEL 1
#define RMX_PHASE_NORMAL 2      /* per-solid counts and the normals of layers <= nl      */
#define RMX_PHASE_EXTRAP 3      /* + (layer - 1), layers 1..RMX_MAX_LAYERS               */
#define RMX_PHASE_BAND 19       /* the persistent band launch (RMX_FLAG_PERSISTENT)       */
#define RMX_PHASE_STEP_TRANS 20   /* rmx_step: transverse face states                     */
#define RMX_PHASE_STEP_PREDICT 21 /* rmx_step: predictor and the interior mask at n + 1   */
#define RMX_PHASE_STEP_CORRECT 22 /* rmx_step: corrector                                  */
#define RMX_PHASE_STEP_FACES 23   /* rmx_step: chosen xi states on the faces              */
#define RMX_N_PHASES 24

/* Grid: M x N x O cells (SI, "Variable arrangement").  Cell (i,j,k) has centre
 * origin + (idx + 1/2) Delta with Delta_a = spacing[a], or h where spacing[a] is 0 (all
 * zero: isotropic spacing h, as in the paper's runs).  The extrapolation sees only the
 * ratios of the spacings: with unequal ones the normal factor of eq. (weight) is the
 * cosine between the physical offset (dx Delta_x, dy Delta_y, dz Delta_z) and the
 * physical gradient of phi0(xi); the fit itself stays in cell offsets (its value at the
 * target does not depend on the scale of its columns).  rmx_step advects with
 * dt / Delta_a per axis and rmx_solid_stress differentiates with Delta_a.
 * periodic[a] != 0: the grid wraps along axis a (SI "Test cases": periodic boxes).  A
 * solid's box then holds its unwrapped map: 0 <= lo[a] < n[a] and ext[a] <= n[a], and the
 * box may run past n[a] (its local cell l lies on grid cell (lo + l) mod n).  No box face
 * along a periodic axis is a wall, so a band that reaches one is truncated.  Zero-fill
 * the struct before setting fields (reserved must be 0). */
typedef struct {
    int32_t n[3];
    double h;
    double origin[3];
    double spacing[3];
    int32_t periodic[3];
    int32_t reserved;
} rmx_grid;

/* phi0 in reference coordinates.  Body coordinates y = rot^T (xi - centre); rot is
 * row-major and orthonormal (columns = body axes).  Sphere: radius semi_axes[0].
 * Ellipsoid: semi-axes along the body axes.  phi0 is the exact signed distance. */
typedef struct {
    int32_t kind;
    double centre[3];
    double semi_axes[3];
    double rot[9];
} rmx_shape;

/* One solid.  Its box D = [lo, lo + ext) must lie in the grid and hold the solid's
 * interior and band.  xi is SoA [3][ext2][ext1][ext0] FP64 (x fastest); a cell with a
 * non-finite component is undefined (never interior).  labels is [ext2][ext1][ext0]:
 * -1 unmarked, 0 interior, 1..L band layer.  decisions (nullable) receives per cell 0
 * (not band), r (fitted with radius r), 32 (F1), 33 (F2), plus 64 if the cell's layer
 * uses the normal but the gradient vanished.  xi_normal (nullable) is the field the
 * normals are taken from (same layout); NULL = xi at the start of the call. */
typedef struct {
    int32_t lo[3];
    int32_t ext[3];
    rmx_shape phi0;
    int32_t n_layers;
    double* xi;               /* DEVICE, in/out                                          */
    const double* xi_normal;  /* DEVICE, in, nullable                                    */
    int8_t* labels;           /* DEVICE, out                                             */
    int8_t* decisions;        /* DEVICE, out, nullable                                   */
} rmx_solid;

/* r_s: search radius (paper: 2); r_max: growth cap (>= r_s, <= RMX_MAX_RADIUS);
 * normal_layers: layers that use the normal factor (paper: 2); precision RMX_FP64 or
 * RMX_FP32_ACCUM (FP32 gathers and moments, FP64 solve and update). */
typedef struct {
    int32_t r_s;
    int32_t r_max;
    int32_t normal_layers;
    int32_t precision;
    uint32_t flags;
} rmx_options;

typedef struct {
    int64_t n_interior;
    int64_t n_band[RMX_MAX_LAYERS + 1];   /* n_band[l], l = 1..L; n_band[0] unused      */
    int64_t n_r_grown;                    /* cells fitted at r > r_s, or by F1/F2        */
    int64_t n_no_normal;
    int64_t n_f1;
    int64_t n_f2;
    int32_t status;                       /* RMX_OK, RMX_W_EMPTY or RMX_E_TRUNCATED      */
    int32_t pad_;
} rmx_solid_stats;

typedef struct rmx_ctx rmx_ctx;
typedef struct rmx_server rmx_server;

/* Fill *opt with the paper's settings: r_s = 2, r_max = 4, normal_layers = 2, FP64. */
int rmx_default_options(rmx_options* opt);

/* Create a context on HIP device `device`.  workspace_bytes = 0: the workspace grows on
 * demand (a growth frees the old workspace, which waits for the device); > 0: allocated
 * once, and calls needing more fail with RMX_E_WORKSPACE. */
int rmx_create(int device, size_t workspace_bytes, rmx_ctx** out);
int rmx_destroy(rmx_ctx* ctx);

/* Workspace bytes a call with these arguments needs (about 25 bytes per box cell with
 * normals, 1 without); the field pointers of `solids` are not used. */
int rmx_workspace_size(const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
                       const rmx_options* opt, size_t* bytes);

/* Extrapolate n_solids solids, each independently, enqueued on `hip_stream` (a
 * hipStream_t; NULL = the default stream).  Arguments are validated on the host first
 * (nothing is enqueued on error).  By default the whole batch runs as one chain of
 * kernels, each covering every solid (classify, label, normals, one fit per layer);
 * RMX_FLAG_PERSISTENT puts the normals and every layer's fits in one persistent launch;
 * RMX_FLAG_PER_SOLID runs one chain per solid instead (the plain form).  Calls on one context are ordered
 * on its workspace: issue them on one stream (or serialise them).
 * If `stats` (HOST, n_solids entries) is non-NULL or
 * RMX_FLAG_SYNC is set, the call waits for the stream, fills `stats` and returns the
 * first negative per-solid status (else RMX_OK); otherwise it returns at once and the
 * call does not allocate once the workspace suffices (graph-capturable). */
int rmx_extrapolate(rmx_ctx* ctx, const rmx_grid* grid, const rmx_solid* solids,
                    int32_t n_solids, const rmx_options* opt, void* hip_stream,
                    rmx_solid_stats* stats);

/* Allocation-free variant of rmx_extrapolate, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and statuses as rmx_extrapolate (the same kernels),
 * but the workspace is a fixed array of 64 MiB per device, reserved in the library's
 * device code and held until the process ends, and nothing is allocated: no device,
 * pinned or graph memory.  Limits, checked on the host before anything is enqueued:
 * the call's workspace (rmx_workspace_size, about 25 B per box cell with normals) must
 * not exceed 64 MiB and its descriptors 256 KiB, else RMX_E_WORKSPACE; with `stats` or
 * RMX_FLAG_SYNC at most 4096 solids (else RMX_E_WORKSPACE); RMX_FLAG_GRAPH and
 * RMX_FLAG_PROFILE are refused (RMX_E_ARG).  Every such call on one device shares that
 * device's array, which keeps the last call's contents; calls that overlap on one device
 * (other contexts, other streams, other host threads) race on it and must be serialised
 * by the caller. */
int rmx_extrapolate_noalloc(rmx_ctx* ctx, const rmx_grid* grid, const rmx_solid* solids,
                            int32_t n_solids, const rmx_options* opt, void* hip_stream,
                            rmx_solid_stats* stats);

/* ---- one time step around the extrapolation ------------------------------------------
 * SI "Timestepping algorithm", steps 5, 6, 7 and 11, with SI "Evaluating the advective
 * term" (eq. (adv_terms); the Taylor-expanded face states of xi; the Godunov-type
 * upwinding scheme; Colella's fourth-order monotonicity-limited normal slopes; upwinded
 * tangential derivatives):
 *   5. predictor xi^{n+1} = xi^n - dt [(u.grad) xi]^{n+1/2} (eq. (dis_xi_adv)) on every
 *      cell labelled 0..L-4 at step n that is at least 3 cells inside the box (its face
 *      states read only defined maps of the labelled band: the stencil reaches 3 cells
 *      along an axis, L1 distance 4); the rest of the old band (labels 0..L at n) becomes
 *      undefined (NaN); other cells of xi_next are left as they are;
 *   6. extrapolation from the predicted interior (cells above with phi0(xi^{n+1}) < 0) into
 *      layers 1..L, exactly as rmx_extrapolate, into xi_next / labels_next / decisions;
 *   7. corrector xi_half = (xi^n + xi^{n+1}) / 2 on cells labelled at n + 1 that were
 *      labelled at n, xi^{n+1} on cells labelled only at n + 1; others left as they are;
 *  11. restoring xi^{n+1} is the caller keeping xi_next (swap xi_n <-> xi_next and
 *      labels_n <-> labels_next for the next step: no copy).
 * Readings: the face state of xi is chosen by the sign of the given face-normal velocity,
 * which also advects (the caller's MAC velocity at n + 1/2); the transverse expansions use
 * the cell velocity u^n and its own limited slope.  Lengths: dt and grid->h; velocities in
 * length per time.  Requires L >= 5 (so that cells entering the solid, labelled <= 1 at
 * step n, are predicted).  An interior cell of step n closer than 3 cells to a box face
 * cannot be predicted: the solid reports RMX_E_TRUNCATED (its labels at n + 1 are
 * written, its band and xi_half are not), as does a band that would leave the box.
 * Layouts: xi_n, u, xi_next, xi_half SoA [3][ext2][ext1][ext0] FP64; labels [ext2][ext1]
 * [ext0] int8; uf[0] [ext2][ext1][ext0+1] (x-faces, face i between cells i-1 and i),
 * uf[1] [ext2][ext1+1][ext0], uf[2] [ext2+1][ext1][ext0].  All DEVICE, caller-owned; the
 * inputs are read only; xi_n must not alias xi_next or xi_half. */
typedef struct {
    int32_t lo[3];
    int32_t ext[3];
    rmx_shape phi0;
    int32_t n_layers;         /* L >= 5                                                   */
    const double* xi_n;       /* DEVICE, in: xi^n, defined where labels_n is 0..L          */
    const int8_t* labels_n;   /* DEVICE, in: labels of step n                              */
    const double* u;          /* DEVICE, in: cell-centred velocity u^n                     */
    const double* uf[3];      /* DEVICE, in: face-normal velocities at n + 1/2             */
    double* xi_next;          /* DEVICE, out: xi^{n+1} (predictor + extrapolated band)     */
    int8_t* labels_next;      /* DEVICE, out: labels of step n + 1                         */
    double* xi_half;          /* DEVICE, out: xi^{n+1/2}                                   */
    int8_t* decisions;        /* DEVICE, out, nullable: as for rmx_extrapolate             */
} rmx_step_solid;

/* One time step of every solid of the batch, enqueued on hip_stream as one chain (four
 * step kernels around the extrapolation's label, normal and layer-fit launches; no
 * classification pass: the predictor writes the interior mask).  dt > 0, finite.  Options
 * as for rmx_extrapolate (RMX_FLAG_SYNC, RMX_FLAG_PROFILE, precision, radii, normal
 * layers); RMX_FLAG_GRAPH, RMX_FLAG_PER_SOLID and RMX_FLAG_PERSISTENT are RMX_E_ARG.
 * stats (HOST, nullable, n_solids entries) implies a wait, as for rmx_extrapolate.  The
 * step's own workspace holds 240 B per box cell (transverse face states and the
 * expansions to the faces), on top of the extrapolation's. */
int rmx_step(rmx_ctx* ctx, const rmx_grid* grid, const rmx_step_solid* solids,
             int32_t n_solids, const rmx_options* opt, double dt, void* hip_stream,
             rmx_solid_stats* stats);

/* ---- blur-zone consumers of the extrapolated maps -------------------------------------
 * Main text, "Blurred interface method and monolithic governing equations": phi = phi0(xi)
 * and the smoothed Heaviside H_eps of eq. (sm_heavi); SI "Stress calculations": the
 * neo-Hookean solid stress at cell faces and the multi-body modified Heaviside of
 * eq. (mod_heaviside).  Inputs are the solids as an extrapolation call left them (xi and
 * labels of each box: a solid covers the cells it labels 0..L; its blur zone must lie in
 * its band, i.e. L h > eps).  Both calls are asynchronous on hip_stream.  Sums over solids
 * run in increasing solid index.
 *
 * rmx_blur: on every grid cell inside some box, H = max(1 - sum_m (1 - H_eps(phi_m)), 0)
 * into H (DEVICE, [n2][n1][n0] of the grid, nullable); cells outside every box are left
 * as they are (pure fluid: the caller sets them to 1 once).  phi (HOST array of n_solids
 * DEVICE pointers, nullable, entries nullable): phi_m on the cells of box m labelled 0..L.
 *
 * rmx_solid_stress: on every face with a cell inside some box (faces normal to axis a in
 * tau[a], DEVICE, [6][n2 + (a==2)][n1 + (a==1)][n0 + (a==0)], components xx, yy, zz, xy,
 * xz, yz): per solid m whose difference stencil at the face is labelled (the two cells,
 * and their neighbours across both other axes), grad xi at the face (the difference across
 * the face, the mean of the two cells' centred differences along the other axes),
 * F = (grad xi)^{-1}, B = F F^T, tau_m = G[m] (B - tr(B)/3 I), weight
 * w_m = 1 - H_eps(phi0_m((xi(P) + xi(Q)) / 2)); the face gets T = sum w_m tau_m if
 * S = sum w_m <= 1, else T / S (zero where no solid contributes).  G: HOST, n_solids
 * shear moduli. */
int rmx_blur(rmx_ctx* ctx, const rmx_grid* grid, const rmx_solid* solids, int32_t n_solids,
             double eps, double* H, double* const* phi, void* hip_stream);
int rmx_solid_stress(rmx_ctx* ctx, const rmx_grid* grid, const rmx_solid* solids,
                     int32_t n_solids, double eps, const double* G, double* const* tau,
                     void* hip_stream);

/* Layers for a blur zone ("Extrapolation of xi", first paragraph: L is chosen so that the
 * band covers the whole blur zone).  Host only.  *L = the smallest layer count that labels
 * every cell with phi < eps around a resolved solid (one that holds a ball of radius
 * sqrt(3) h / 2 beneath every surface point), plus `reach` further layers for the
 * consumer's stencil: a cell with 0 < phi < eps lies within physical distance
 * stretch * eps of the surface (stretch >= 1 bounds physical over reference lengths;
 * 1 for an undeformed map), hence within D = stretch * eps + sqrt(3) h of an interior
 * cell centre, i.e. within ceil(D / h) layers of the 26-neighbour adjacency
 * (RMX_FLAG_ADJ26 in flags) or ceil(sqrt(3) D / h) face layers.  h: the grid spacing
 * (equal on the three axes).  RMX_E_ARG for non-positive or non-finite arguments or reach < 0;
 * RMX_E_LAYERS if the count exceeds RMX_MAX_LAYERS. */
int rmx_layers_for_blur(double eps, double h, double stretch, int32_t reach, uint32_t flags,
                        int32_t* L);

/* The same count on a grid with unequal spacings (rmx_grid.spacing; equal spacings give
 * rmx_layers_for_blur's count with h).  Host only.  With Delta_a the spacings, a resolved
 * solid holds a ball of radius |Delta| / 2 beneath every surface point, so a cell with
 * 0 < phi < eps lies within D = stretch * eps + |Delta| of an interior cell centre; that
 * is at most ceil(D / min_a Delta_a) cube layers (RMX_FLAG_ADJ26) or
 * ceil(D * sqrt(sum_a Delta_a^-2)) face layers (the L1 cell distance of a displacement v
 * is sum_a |v_a| / Delta_a <= |v| sqrt(sum_a Delta_a^-2)), plus `reach`.  Errors as
 * rmx_layers_for_blur's, and RMX_E_ARG for a null or invalid grid. */
int rmx_layers_for_blur_grid(const rmx_grid* grid, double eps, double stretch, int32_t reach,
                             uint32_t flags, int32_t* L);

const char* rmx_status_string(int status);

/* Autotuner.  Launch shapes that change no result: the label tile width (1, 2 or 4 words
 * of 64 cells) and the number of blocks striding over a layer's brick list.  rmx_autotune
 * times every candidate over `reps` calls of this batch on `hip_stream` (each candidate on
 * the same input: xi is saved first and restored before each candidate and at the end;
 * labels and decisions hold the last timed call's result), keeps the fastest for later
 * calls of the same shape class on this context (same largest layer count, row width,
 * normal layers and size class), and returns it in *best (HOST).  It allocates (a copy of
 * xi) and synchronises: a set-up call, not for graph capture. */
typedef struct {
    int32_t tile_w;
    int32_t extrap_blocks;
    double ms;                /* average time of one call with this shape */
} rmx_tuning;
int rmx_autotune(rmx_ctx* ctx, const rmx_grid* grid, const rmx_solid* solids,
                 int32_t n_solids, const rmx_options* opt, void* hip_stream, int32_t reps,
                 rmx_tuning* best);

/* Keep launch shapes `t` (HOST; t->ms is ignored) for later calls of this batch's shape
 * class on this context, as rmx_autotune would after choosing them, without timing
 * anything: a shape found by an earlier autotuner run, or one fixed for a profile.
 * tile_w must be 1, 2 or 4 and fit the LDS for this batch's layer count (else RMX_E_ARG);
 * extrap_blocks >= 1.  Allocates nothing on the device. */
int rmx_set_tuning(rmx_ctx* ctx, const rmx_grid* grid, const rmx_solid* solids,
                   int32_t n_solids, const rmx_options* opt, const rmx_tuning* t);

/* Profiling (tracing): wait for every call made with RMX_FLAG_PROFILE since the last
 * read, then write per phase the summed kernel time in ms (ms[RMX_N_PHASES], HOST) and
 * the number of launches (launches[RMX_N_PHASES], HOST), and reset the sums. */
int rmx_profile_read(rmx_ctx* ctx, double* ms, int64_t* launches);

/* ---- serving ------------------------------------------------------------------------
 * A request loop for many concurrently running simulations (object independence, main
 * text "Extrapolation of xi", third paragraph, makes every request independent).
 * register: the server allocates the simulation's resident fields (xi, labels) in HBM
 *   against the budget; fill them through rmx_server_field.  Returns RMX_E_BUDGET if
 *   the fields alone exceed the budget.
 * submit: non-blocking; queues one extrapolation of all solids of the simulation.  A
 *   scheduler thread admits queued requests while their workspace fits the budget left
 *   (continuous batching: requests arriving while others run join the next launch round
 *   as memory frees up), groups them into batched launches over `n_streams` streams.
 * wait: blocks until the ticket completes; returns its status and latency (seconds from
 *   submit to completion).  A request that can never fit fails with RMX_E_BUDGET alone.
 */
int rmx_server_create(int device, size_t hbm_budget_bytes, int32_t n_streams,
                      rmx_server** out);
int rmx_server_register(rmx_server* srv, const rmx_grid* grid, const rmx_solid* templ,
                        int32_t n_solids, int64_t* sim_id);
int rmx_server_field(rmx_server* srv, int64_t sim_id, int32_t solid, double** xi,
                     int8_t** labels);
int rmx_server_submit(rmx_server* srv, int64_t sim_id, const rmx_options* opt,
                      int64_t* ticket);
int rmx_server_wait(rmx_server* srv, int64_t ticket, rmx_solid_stats* stats,
                    double* latency_s);
int rmx_server_release(rmx_server* srv, int64_t sim_id);
/* bytes currently admitted (resident fields + in-flight workspace) and the peak seen */
int rmx_server_usage(rmx_server* srv, size_t* in_use, size_t* peak);
int rmx_server_destroy(rmx_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* RMX_H */
